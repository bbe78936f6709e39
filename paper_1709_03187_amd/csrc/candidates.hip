// Candidate lists, spatial grid and pheromone initialisation.
//
// The pheromone lives only on each city's k nearest neighbours (the
// candidate-list device of ACS, recalled in Section 6 of the paper), so the
// store is n x k instead of the n x n matrix Section 3 rules out at 100K+
// cities.  A uniform grid with about two cities per cell serves both the
// k-NN build and the exact nearest-unvisited fallback.
#include <cmath>
#include <cstring>

#include "colony.hpp"
#include "common.hpp"

namespace aco {

// ------------------------------------------------------------------ grid build

// bbox[0..3] = min x, min y, max x, max y; bbox[4] = 1 if a coordinate is out of range.
__global__ void k_bbox_init(int32_t *bbox)
{
    if (threadIdx.x == 0) {
        bbox[0] = INT32_MAX;
        bbox[1] = INT32_MAX;
        bbox[2] = INT32_MIN;
        bbox[3] = INT32_MIN;
        bbox[4] = 0;
    }
}

__global__ void k_bbox(const int32_t *__restrict__ xy, int32_t n, int32_t *bbox)
{
    int32_t mnx = INT32_MAX, mny = INT32_MAX, mxx = INT32_MIN, mxy = INT32_MIN, bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = xy[2 * i], y = xy[2 * i + 1];
        mnx = min(mnx, x);
        mny = min(mny, y);
        mxx = max(mxx, x);
        mxy = max(mxy, y);
        bad |= (x > ACO_COORD_LIMIT || x < -ACO_COORD_LIMIT || y > ACO_COORD_LIMIT ||
                y < -ACO_COORD_LIMIT);
    }
    for (int off = 32; off > 0; off >>= 1) {
        mnx = min(mnx, __shfl_xor(mnx, off));
        mny = min(mny, __shfl_xor(mny, off));
        mxx = max(mxx, __shfl_xor(mxx, off));
        mxy = max(mxy, __shfl_xor(mxy, off));
        bad |= __shfl_xor(bad, off);
    }
    if (lane_id() == 0) {
        atomicMin(&bbox[0], mnx);
        atomicMin(&bbox[1], mny);
        atomicMax(&bbox[2], mxx);
        atomicMax(&bbox[3], mxy);
        if (bad) atomicOr(&bbox[4], 1);
    }
}

__global__ void k_write_hdr(GridHdr h, void *grid)
{
    if (threadIdx.x == 0) *(GridHdr *)grid = h;
}

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_grid_count(const int32_t *__restrict__ xy, GridHdr h, int32_t *count)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= h.n) return;
    const int c = cell_y(h, xy[2 * i + 1]) * h.gw + cell_x(h, xy[2 * i]);
    atomicAdd(&count[c], 1);
}

// In-place exclusive scan of v[0..len) by one workgroup of 1024 threads, each
// owning a contiguous strip; cursor receives a copy of the result.
__global__ __launch_bounds__(1024) void k_scan_excl(int32_t *v, int32_t *cursor, int64_t len)
{
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int64_t strip = (len + 1023) / 1024;
    const int64_t lo = min(len, t * strip), hi = min(len, lo + strip);
    int32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += v[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t add = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int32_t run = part[t] - s;
    for (int64_t i = lo; i < hi; ++i) {
        const int32_t c = v[i];
        v[i] = run;
        cursor[i] = run;
        run += c;
    }
}

__global__ void k_grid_scatter(const int32_t *__restrict__ xy, GridHdr h, int32_t *cursor,
                               int4 *pts, int32_t *pinv)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= h.n) return;
    const int32_t x = xy[2 * i], y = xy[2 * i + 1];
    const int c = cell_y(h, y) * h.gw + cell_x(h, x);
    const int pos = atomicAdd(&cursor[c], 1);
    pts[pos] = make_int4(x, y, (int)i, 0);
    pinv[i] = pos;
}

// ------------------------------------------------------------------ k-NN build

// One thread per city, cities taken in grid order so that a wave works on
// neighbouring cities.  Each thread scans rings of cells of growing radius
// around its city and keeps the kxp smallest keys (d, j) in an LDS heap
// (interleaved by thread to avoid bank conflicts); it stops once every point
// outside the searched block is farther than the kxp-th distance.
// The candidate list (k), the table by city (kx) and the table by position
// (kxp) are prefixes of that list.  32 threads: a 256-entry list per thread
// fits the workgroup's 64 KB.
constexpr int kKnnThreads = 32;

__global__ __launch_bounds__(kKnnThreads) void k_knn(void *grid, int32_t k, int32_t *nn,
                                                      int32_t *nnd)
{
    extern __shared__ uint64_t lists[];   // [kxp][kKnnThreads]
    const GridView g = grid_view(grid);
    const int kx = g.h.kx, kxp = g.h.kxp;   // k <= kx <= kxp
    int32_t *ext = (int32_t *)g.ext;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= g.h.n) return;
    uint64_t *L = lists + threadIdx.x;
    const int4 me = g.pts[p];
    knn_city_wide(g, me, kxp, L, kKnnThreads);
    const int64_t row = (int64_t)me.z * k, xrow = (int64_t)me.z * kx, prow = p * kxp;
    int32_t *ext_pos = (int32_t *)g.ext_pos;
    for (int r = 0; r < kxp; ++r) {
        const uint64_t key = L[(int64_t)r * kKnnThreads];
        ext_pos[prow + r] = g.pinv[(uint32_t)key];
        if (r < kx) ext[xrow + r] = (int32_t)(uint32_t)key;
        if (r < k) {
            nn[row + r] = (int32_t)(uint32_t)key;
            nnd[row + r] = (int32_t)(key >> 32);
        }
    }
}

// rev[i][r] = position of i in nn[nn[i][r]], -1 if absent.
__global__ void k_rev(const int32_t *__restrict__ nn, int32_t n, int32_t k, int8_t *rev)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * k) return;
    const int32_t i = (int32_t)(e / k);
    const int32_t j = nn[e];
    int8_t out = -1;
    for (int s = 0; s < k; ++s)
        if (nn[(int64_t)j * k + s] == i) {
            out = (int8_t)s;
            break;
        }
    rev[e] = out;
}

// eta_b = fl32(eta^beta), eta = 1/max(d,1) or a supplied score, in FP64.
__global__ void k_eta(const int32_t *__restrict__ nnd, const float *__restrict__ eta_in,
                      int64_t count, double beta, float *eta_b)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= count) return;
    double eta;
    if (eta_in) {
        eta = (double)eta_in[e];
    } else {
        const int32_t d = nnd[e];
        eta = 1.0 / (double)(d > 1 ? d : 1);
    }
    eta_b[e] = (float)(beta == 0.0 ? 1.0 : (beta == 1.0 ? eta : pow(eta, beta)));
}

// ------------------------------------------------------------------ NN tour

// The nearest-neighbour tour from city 0 by one wave on cell-order positions
// (the visited bits are the workgroup's LDS).  nn and nnd are not needed: the
// grid's 64-NN table by position starts with the candidate list.

// The two-hop table (one thread per entry): row c, group q holds the first 16
// entries of the neighbour row of c (q = 0) or of c's q-th nearest neighbour.
__global__ void k_nn_hop(const void *grid, int32_t n, int32_t *hop)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * kHopWidth) return;
    const GridView g = grid_view(grid);
    const int64_t c = t / kHopWidth;
    const int e = (int)(t % kHopWidth), q = e / 16, r = e % 16;
    const int kf = g.h.kxp < 16 ? g.h.kxp : 16;
    int32_t v = -1;
    if (r < kf && q - 1 < kf) {
        const int64_t row = q == 0 ? c : (int64_t)g.ext_pos[c * g.ext_pos_stride + (q - 1)];
        v = g.ext_pos[row * g.ext_pos_stride + r];
    }
    hop[t] = v;
}

__global__ __launch_bounds__(kWave) void k_nn_tour_hop(int32_t n, const void *grid,
                                                      const int32_t *hop, int32_t *tour,
                                                      uint32_t *err)
{
    extern __shared__ uint32_t vis[];
    nn_tour_positions_hop(grid_view(grid), n, VisBits{vis}, hop, tour, err);
}

// Closed length of one tour by one workgroup of 256 threads (exact integer
// sum; the order of the additions does not matter).
__global__ __launch_bounds__(256) void k_closed_length(const int32_t *__restrict__ xy,
                                                       const int32_t *__restrict__ tour,
                                                       int32_t n, int64_t *length)
{
    __shared__ int64_t part[256 / kWave];
    int64_t s = 0;
    for (int32_t t = threadIdx.x; t < n; t += blockDim.x) {
        const int64_t a = tour[t], b = tour[t + 1 < n ? t + 1 : 0];
        s += nint_sqrt(sq_dist(xy[2 * a], xy[2 * a + 1], xy[2 * b], xy[2 * b + 1]));
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += part[w];
        *length = t;
    }
}

__global__ void k_fill_f32(float *p, int64_t count, float v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------------ host side

static int64_t isqrt_ceil_i64(int64_t v)
{
    if (v <= 0) return 0;
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r > 0 && (r - 1) * (r - 1) >= v) --r;
    while (r * r < v) ++r;
    return r;
}

// Builds the grid in `grid`; the bounding box is read back to size the cells.
int build_grid(const int32_t *xy, int32_t n, void *grid, size_t grid_bytes, hipStream_t st)
{
    const GridLayout lay(n);
    if (grid_bytes < lay.total)
        return fail(ACO_ERR_WORKSPACE, "grid buffer has %zu bytes, needs %zu", grid_bytes,
                    lay.total);
    char *gb = (char *)grid;
    int32_t *scratch = (int32_t *)(gb + lay.cursor);
    k_bbox_init<<<1, 64, 0, st>>>(scratch);
    k_bbox<<<min(1024u, blocks_for(n, 256)), 256, 0, st>>>(xy, n, scratch);
    ACO_LAUNCH_CHECK("k_bbox");
    int32_t bb[5];
    ACO_HIP_CHECK(hipMemcpyAsync(bb, scratch, sizeof(bb), hipMemcpyDeviceToHost, st));
    ACO_HIP_CHECK(hipStreamSynchronize(st));
    if (bb[4]) return fail(ACO_ERR_INVALID_ARG, "a coordinate exceeds +-%d", ACO_COORD_LIMIT);
    if (bb[0] == bb[2] && bb[1] == bb[3])
        return fail(ACO_ERR_DEGENERATE, "all %d cities coincide", n);
    const int64_t W = (int64_t)bb[2] - bb[0] + 1, H = (int64_t)bb[3] - bb[1] + 1;
    const int64_t target = n / 2 > 0 ? n / 2 : 1;
    // cell side: about two cities per cell, and at most n cells along either side
    int64_t cell = isqrt_ceil_i64((W * H + target - 1) / target);
    cell = std::max<int64_t>(cell, (std::max(W, H) + n - 1) / n);
    cell = std::max<int64_t>(cell, 1);
    GridHdr h;
    h.x0 = bb[0];
    h.y0 = bb[1];
    h.cell = (int32_t)cell;
    h.gw = (int32_t)((W + cell - 1) / cell);
    h.gh = (int32_t)((H + cell - 1) / cell);
    h.ncell = h.gw * h.gh;
    h.n = n;
    h.cap = (int32_t)GridLayout::cap_for(n);
    h.kx = ext_width(n);
    h.kxp = ext_pos_width(n);
    if ((int64_t)h.gw * h.gh + 1 > h.cap)
        return fail(ACO_ERR_HIP, "grid sizing error (%d x %d cells)", h.gw, h.gh);
    int32_t *cell_start = (int32_t *)(gb + lay.cell_start);
    int32_t *cursor = (int32_t *)(gb + lay.cursor);
    int4 *pts = (int4 *)(gb + lay.pts);
    int32_t *pinv = (int32_t *)(gb + lay.pinv);
    k_write_hdr<<<1, 64, 0, st>>>(h, grid);
    k_fill_i32<<<min(4096u, blocks_for(h.ncell + 1, 256)), 256, 0, st>>>(cell_start,
                                                                        h.ncell + 1, 0);
    k_grid_count<<<blocks_for(n, 256), 256, 0, st>>>(xy, h, cell_start);
    k_scan_excl<<<1, 1024, 0, st>>>(cell_start, cursor, (int64_t)h.ncell + 1);
    k_grid_scatter<<<blocks_for(n, 256), 256, 0, st>>>(xy, h, cursor, pts, pinv);
    ACO_LAUNCH_CHECK("grid build");
    return ACO_OK;
}

}  // namespace aco

using namespace aco;

extern "C" size_t aco_grid_bytes(int32_t n)
{
    return n < 1 ? 0 : GridLayout(n).total;
}

extern "C" int aco_build_candidates(const int32_t *xy, int32_t n, int32_t k, double beta,
                                    const float *eta, int32_t *nn, int32_t *nnd, int8_t *rev,
                                    float *eta_b, void *grid, size_t grid_bytes, void *stream)
{
    clear_error();
    ACO_REQUIRE(n >= 3 && n <= (1 << 27), "n = %d out of range [3, 2^27]", n);
    ACO_REQUIRE(k >= 1 && k <= ACO_MAX_K && k <= n - 1, "k = %d out of range [1, min(n-1, %d)]",
                k, ACO_MAX_K);
    ACO_REQUIRE(std::isfinite(beta) && beta >= 0.0, "beta must be finite and >= 0");
    ACO_REQUIRE(xy && nn && nnd && rev && eta_b && grid, "NULL array argument");
    hipStream_t st = as_stream(stream);
    int rc = build_grid(xy, n, grid, grid_bytes, st);
    if (rc != ACO_OK) return rc;
    const size_t lds = (size_t)ext_pos_width(n) * kKnnThreads * sizeof(uint64_t);
    if (lds > max_lds_per_block())
        return fail(ACO_ERR_UNSUPPORTED, "neighbour lists of %zu bytes exceed LDS (%zu)", lds,
                    max_lds_per_block());
    if (lds > 65536)
        ACO_HIP_CHECK(hipFuncSetAttribute((const void *)k_knn,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    k_knn<<<blocks_for(n, kKnnThreads), kKnnThreads, lds, st>>>(grid, k, nn, nnd);
    ACO_LAUNCH_CHECK("k_knn");
    const int64_t nk = (int64_t)n * k;
    k_rev<<<blocks_for(nk, 256), 256, 0, st>>>(nn, n, k, rev);
    k_eta<<<blocks_for(nk, 256), 256, 0, st>>>(nnd, eta, nk, beta, eta_b);
    ACO_LAUNCH_CHECK("k_rev/k_eta");
    return ACO_OK;
}

extern "C" int aco_init_pheromone(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                                  const int32_t *nnd, void *grid, int32_t *nn_tour, float *tau,
                                  float *tau0_out, int64_t *L_nn_out, void *stream)
{
    clear_error();
    ACO_REQUIRE(n >= 3 && n <= (1 << 27), "n = %d out of range [3, 2^27]", n);
    ACO_REQUIRE(k >= 1 && k <= ACO_MAX_K && k <= n - 1, "k = %d out of range", k);
    ACO_REQUIRE(xy && nn && nnd && grid && nn_tour && tau, "NULL array argument");
    const size_t lds = bitmask_bytes(n);
    if (lds > max_lds_per_block())
        return fail(ACO_ERR_UNSUPPORTED, "visited bitmask of %zu bytes exceeds LDS (%zu)", lds,
                    max_lds_per_block());
    hipStream_t st = as_stream(stream);
    int64_t *dlen = (int64_t *)((char *)grid + GridLayout::kAuxOffset);
    if (lds > 65536)
        ACO_HIP_CHECK(hipFuncSetAttribute((const void *)k_nn_tour_hop,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    uint32_t *err = device_error_word();
    if (!err) return ACO_ERR_HIP;
    // the two-hop table lives in stream-ordered scratch for the tour only
    int32_t *hop = nullptr;
    const size_t hop_bytes = (size_t)n * kHopWidth * sizeof(int32_t);
    ACO_HIP_CHECK(hipMallocAsync((void **)&hop, hop_bytes, st));
    const int64_t entries = (int64_t)n * kHopWidth;
    k_nn_hop<<<blocks_for(entries, 256), 256, 0, st>>>(grid, n, hop);
    hipError_t le = hipGetLastError();
    if (le == hipSuccess) {
        k_nn_tour_hop<<<1, kWave, lds, st>>>(n, grid, hop, nn_tour, err);
        le = hipGetLastError();
    }
    // the scratch is released whether or not the launches went through
    const hipError_t fe = hipFreeAsync(hop, st);
    if (le != hipSuccess)
        return fail(ACO_ERR_HIP, "launch of the NN tour failed: %s", hipGetErrorString(le));
    if (fe != hipSuccess) return fail(ACO_ERR_HIP, "hipFreeAsync failed");
    k_closed_length<<<1, 256, 0, st>>>(xy, nn_tour, n, dlen);
    ACO_LAUNCH_CHECK("k_closed_length");
    int64_t L = 0;
    ACO_HIP_CHECK(hipMemcpyAsync(&L, dlen, 8, hipMemcpyDeviceToHost, st));
    ACO_HIP_CHECK(hipStreamSynchronize(st));
    const int rc = report_device_error(st);
    if (rc != ACO_OK) return rc;
    if (L <= 0)
        return fail(ACO_ERR_DEGENERATE, "nearest-neighbour tour has length %lld", (long long)L);
    const float t0 = (float)(1.0 / ((double)n * (double)L));
    const int64_t nk = (int64_t)n * k;
    k_fill_f32<<<min(4096u, blocks_for(nk, 256)), 256, 0, st>>>(tau, nk, t0);
    ACO_LAUNCH_CHECK("k_fill_f32");
    if (tau0_out) *tau0_out = t0;
    if (L_nn_out) *L_nn_out = L;
    return ACO_OK;
}
