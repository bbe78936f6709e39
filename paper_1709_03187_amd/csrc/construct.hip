// Tour construction with the random proportional rule (Section 2, Eq. 1).
//
// One ant per 64-wide wavefront.  Per step the ant at city c reads the packed
// candidate row {nn[c][r], w[c][r]} (one 128-byte line at k = 16), tests the
// candidates against its visited bitmask in LDS, forms the FP64 running sum of
// the unvisited weights across lanes, and picks the first lane whose running
// sum exceeds u * S with a ballot.  When no unvisited candidate has positive
// weight the whole wave searches the grid for the nearest unvisited city.
#include <cmath>

#include "common.hpp"
#include "device.hpp"

namespace aco {

// Packed candidate row element: candidate city and its choice weight bits.
struct CandW {
    int32_t city;
    float w;
};

// Choice weights w[i][r] = tau^alpha * eta_b scaled per row by a power of two
// (probabilities are invariant to a per-row factor).  For alpha = 1 the value
// is the exact product tau * eta_b rounded once to FP32 (times 2^E); for other
// alpha it is exp2(alpha log2 tau + log2 eta_b - max over the row).
__global__ void k_choice_info(const int32_t *__restrict__ nn, const float *__restrict__ tau,
                              const float *__restrict__ eta_b, int32_t n, int32_t k, double alpha,
                              CandW *__restrict__ rows)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t rb = i * k;
    if (alpha == 1.0 || alpha == 0.0) {
        double mx = 0.0;
        for (int r = 0; r < k; ++r) {
            const double p = (alpha == 1.0 ? (double)tau[rb + r] : 1.0) * (double)eta_b[rb + r];
            mx = p > mx ? p : mx;
        }
        const int e = (mx > 0.0) ? -ilogb(mx) : 0;
        for (int r = 0; r < k; ++r) {
            const double p = (alpha == 1.0 ? (double)tau[rb + r] : 1.0) * (double)eta_b[rb + r];
            rows[rb + r] = CandW{nn[rb + r], (float)ldexp(p, e)};
        }
    } else {
        double mx = -INFINITY;
        for (int r = 0; r < k; ++r) {
            const double t = (double)tau[rb + r], eb = (double)eta_b[rb + r];
            const double lw = (t > 0.0 && eb > 0.0) ? alpha * log2(t) + log2(eb) : -INFINITY;
            mx = lw > mx ? lw : mx;
        }
        for (int r = 0; r < k; ++r) {
            const double t = (double)tau[rb + r], eb = (double)eta_b[rb + r];
            const double lw = (t > 0.0 && eb > 0.0) ? alpha * log2(t) + log2(eb) : -INFINITY;
            rows[rb + r] = CandW{nn[rb + r], (float)((mx > -INFINITY) ? exp2(lw - mx) : 0.0)};
        }
    }
}

struct ConstructArgs {
    const int32_t *xy;
    const CandW *rows;
    const void *grid;
    int32_t n, k;
    int32_t ant0;
    uint32_t iteration;
    uint64_t seed;
    int32_t *tours;
    int64_t *lengths;
    uint8_t *slots;
    float *step_prob;
};

// One ant per wavefront.  Lane r < k holds candidate r of the current city.
// The critical path of a step is: row load -> visited test (LDS) -> DPP scan
// -> ballot -> next row address.  (Touching the candidates' rows ahead of time
// does not help: vector loads complete in order, so the next row load would
// wait for the slowest of those touches.)
// KP is the scan width: the smallest power of two >= k (a template parameter
// so that the per-step code has no branches besides the roulette/fallback).
template <int KP>
__global__ __launch_bounds__(kWave) void k_construct(ConstructArgs A)
{
    extern __shared__ uint32_t vis[];
    const int lane = lane_id();
    const int32_t n = A.n, k = A.k;
    const int32_t a = blockIdx.x;                 // ant within this launch
    const uint32_t ant = (uint32_t)(A.ant0 + a);  // absolute ant index (Philox counter)
    const int nwords = (n + 31) >> 5;
    for (int w = lane; w < nwords; w += kWave) vis[w] = 0u;
    __syncthreads();
    auto visited = [&](int city) { return (vis[city >> 5] >> (city & 31)) & 1u; };

    int32_t *tour_out = A.tours + (int64_t)a * n;
    uint8_t *slot_out = A.slots + (int64_t)a * n;
    float *prob_out = A.step_prob ? A.step_prob + (int64_t)a * n : nullptr;
    const bool want_prob = prob_out != nullptr;

    // lane l holds the Philox word of step (base + l)
    uint32_t rnd = colony_draw(A.seed, A.iteration, ant, (uint32_t)lane);
    const uint32_t x0 = (uint32_t)read_lane_i32((int32_t)rnd, 0);
    const int32_t start = (int32_t)(((uint64_t)x0 * (uint64_t)n) >> 32);
    if (lane == 0) vis[start >> 5] |= 1u << (start & 31);
    __syncthreads();

    int32_t st_city = start;      // staged outputs: lane l holds step (base + l)
    uint32_t st_slot = kNoSlot;
    float st_prob = 1.0f;
    int32_t c = start;
    const bool active = lane < k;
    const int lr = active ? lane : k - 1;   // idle lanes re-read a valid element
    GridView g;
    bool have_grid = false;

    for (int32_t step = 1; step < n; ++step) {
        if ((step & 63) == 0) rnd = colony_draw(A.seed, A.iteration, ant, (uint32_t)(step + lane));
        const CandW e = A.rows[(int64_t)c * k + lr];
        const int32_t j = e.city;
        const uint32_t seen = visited(j);          // every lane reads a valid word
        const bool unv = active && seen == 0u;
        const double wv = (unv && e.w > 0.0f) ? (double)e.w : 0.0;
        const double cum = wave_incl_scan_f64(wv, KP);
        const double S = read_lane_f64(cum, k - 1);
        int32_t jn;
        uint32_t slot;
        float prob = -1.0f;
        if (S > 0.0) {
            const uint32_t x = (uint32_t)read_lane_i32((int32_t)rnd, step & 63);
            const double target = (double)x * 0x1p-32 * S;
            const uint64_t hit = __ballot(wv > 0.0 && target < cum);
            const int f = hit ? __ffsll((unsigned long long)hit) - 1
                              : 63 - __clzll((long long)__ballot(wv > 0.0));
            jn = read_lane_i32(j, f);
            slot = (uint32_t)f;
            if (want_prob) prob = (float)(read_lane_f64(wv, f) / S);
        } else {
            if (!have_grid) {
                g = grid_view(A.grid);
                have_grid = true;
            }
            jn = fallback_city(g, A.xy, c, visited);
            slot = kNoSlot;
        }
        // a city index is always in range here; the clamp only keeps a logic
        // error from turning into an out-of-bounds access (tests see the tour)
        jn = ((uint32_t)jn < (uint32_t)n) ? jn : start;
        if (lane == 0) atomicOr(&vis[jn >> 5], 1u << (jn & 31));
        if (lane == (step & 63)) {
            st_city = jn;
            st_slot = slot;
            st_prob = prob;
        }
        if ((step & 63) == 63 || step == n - 1) {
            const int32_t base = step & ~63;
            if (base + lane <= step) {
                tour_out[base + lane] = st_city;
                slot_out[base + lane] = (uint8_t)st_slot;
                if (want_prob) prob_out[base + lane] = st_prob;
            }
        }
        c = jn;
    }
    if (lane == 0) A.lengths[a] = 0;     // summed by k_tour_length
}

// Tour lengths: one block of 256 threads per (ant, chunk of 256 tour edges),
// exact integer distances, one int64 atomic per block.
constexpr int kLenThreads = 256;

__global__ __launch_bounds__(kLenThreads) void k_tour_length(const int32_t *__restrict__ xy,
                                                             const int32_t *__restrict__ tours,
                                                             int32_t n, int32_t chunks,
                                                             unsigned long long *lengths)
{
    __shared__ int64_t part[kLenThreads / kWave];
    const int32_t a = blockIdx.x / chunks;
    const int32_t t = (blockIdx.x - a * chunks) * kLenThreads + threadIdx.x;
    int64_t d = 0;
    if (t < n) {
        const int32_t *T = tours + (int64_t)a * n;
        const int32_t i = T[t], j = T[t + 1 == n ? 0 : t + 1];
        d = nint_sqrt(sq_dist(xy[2 * (int64_t)i], xy[2 * (int64_t)i + 1], xy[2 * (int64_t)j],
                              xy[2 * (int64_t)j + 1]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);
    if (lane_id() == 0) part[threadIdx.x / kWave] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int w = 0; w < kLenThreads / kWave; ++w) s += part[w];
        atomicAdd(&lengths[a], (unsigned long long)s);
    }
}

}  // namespace aco

using namespace aco;

extern "C" size_t aco_construct_workspace_bytes(int32_t n, int32_t k)
{
    if (n < 1 || k < 1) return 0;
    return (size_t)n * (size_t)k * sizeof(CandW);
}

extern "C" int aco_construct_tours(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                                   const int32_t *nnd, const float *eta_b, const void *grid,
                                   const float *tau, int32_t m, int32_t ant0, double alpha,
                                   uint64_t seed, int64_t iteration, int32_t *tours,
                                   int64_t *lengths, uint8_t *slots, float *step_prob, void *ws,
                                   size_t ws_bytes, void *stream)
{
    clear_error();
    ACO_REQUIRE(n >= 3 && n <= (1 << 27), "n = %d out of range [3, 2^27]", n);
    ACO_REQUIRE(k >= 1 && k <= ACO_MAX_K && k <= n - 1, "k = %d out of range", k);
    ACO_REQUIRE(m >= 1 && ant0 >= 0 && (int64_t)ant0 + m <= INT32_MAX, "bad ant range");
    ACO_REQUIRE(iteration >= 0 && iteration <= (int64_t)UINT32_MAX, "iteration out of range");
    ACO_REQUIRE(std::isfinite(alpha) && alpha >= 0.0, "alpha must be finite and >= 0");
    ACO_REQUIRE(xy && nn && nnd && eta_b && grid && tau && tours && lengths && slots && ws,
                "NULL array argument");
    const size_t need = aco_construct_workspace_bytes(n, k);
    if (ws_bytes < need)
        return fail(ACO_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    const size_t lds = bitmask_bytes(n);
    if (lds > max_lds_per_block())
        return fail(ACO_ERR_UNSUPPORTED, "visited bitmask of %zu bytes exceeds LDS (%zu)", lds,
                    max_lds_per_block());
    hipStream_t st = as_stream(stream);
    CandW *rows = (CandW *)ws;
    k_choice_info<<<blocks_for(n, 256), 256, 0, st>>>(nn, tau, eta_b, n, k, alpha, rows);
    ACO_LAUNCH_CHECK("k_choice_info");
    void (*kern)(ConstructArgs) = k <= 8    ? k_construct<8>
                                  : k <= 16 ? k_construct<16>
                                  : k <= 32 ? k_construct<32>
                                            : k_construct<64>;
    if (lds > 65536)
        ACO_HIP_CHECK(hipFuncSetAttribute((const void *)kern,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ConstructArgs A{xy, rows, grid, n, k, ant0, (uint32_t)iteration, seed,
                    tours, lengths, slots, step_prob};
    kern<<<m, kWave, lds, st>>>(A);
    ACO_LAUNCH_CHECK("k_construct");
    const int32_t chunks = (n + kLenThreads - 1) / kLenThreads;
    k_tour_length<<<(unsigned)((int64_t)m * chunks), kLenThreads, 0, st>>>(
        xy, tours, n, chunks, (unsigned long long *)lengths);
    ACO_LAUNCH_CHECK("k_tour_length");
    return ACO_OK;
}
