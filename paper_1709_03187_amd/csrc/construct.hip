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
    const int32_t *nnd;
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

__global__ __launch_bounds__(kWave) void k_construct(ConstructArgs A)
{
    extern __shared__ uint32_t vis[];
    const int lane = lane_id();
    const int32_t n = A.n, k = A.k;
    const int32_t a = blockIdx.x;                 // ant within this launch
    const uint32_t ant = (uint32_t)(A.ant0 + a);  // absolute ant index (Philox counter)
    const GridView g = grid_view(A.grid);
    const int nwords = (n + 31) >> 5;
    for (int w = lane; w < nwords; w += kWave) vis[w] = 0u;
    __syncthreads();
    auto visited = [&](int city) { return (vis[city >> 5] >> (city & 31)) & 1u; };

    int32_t *tour_out = A.tours + (int64_t)a * n;
    uint8_t *slot_out = A.slots + (int64_t)a * n;
    float *prob_out = A.step_prob ? A.step_prob + (int64_t)a * n : nullptr;

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
    int64_t L = 0;
    int kp = 1;
    while (kp < k) kp <<= 1;

    for (int32_t step = 1; step < n; ++step) {
        if ((step & 63) == 0) rnd = colony_draw(A.seed, A.iteration, ant, (uint32_t)(step + lane));
        const int64_t rb = (int64_t)c * k;
        int32_t j = 0, d = 0;
        float wf = 0.0f;
        if (lane < k) {
            const CandW e = A.rows[rb + lane];
            j = e.city;
            wf = e.w;
            d = A.nnd[rb + lane];
        }
        const bool unv = (lane < k) && !visited(j);
        const double wv = (unv && wf > 0.0f) ? (double)wf : 0.0;
        double cum = wv;
        for (int off = 1; off < kp; off <<= 1) {
            const double t = __shfl_up(cum, off);
            if (lane >= off) cum += t;
        }
        const double S = read_lane_f64(cum, k - 1);
        int32_t jn, dn;
        uint32_t slot;
        float prob;
        if (S > 0.0) {
            const uint32_t x = (uint32_t)read_lane_i32((int32_t)rnd, step & 63);
            const double target = (double)x * 0x1p-32 * S;
            const uint64_t hit = __ballot(wv > 0.0 && target < cum);
            const int f = hit ? __ffsll((unsigned long long)hit) - 1
                              : 63 - __clzll((long long)__ballot(wv > 0.0));
            jn = read_lane_i32(j, f);
            dn = read_lane_i32(d, f);
            slot = (uint32_t)f;
            prob = (float)(read_lane_f64(wv, f) / S);
        } else {
            const int32_t cx = A.xy[2 * (int64_t)c], cy = A.xy[2 * (int64_t)c + 1];
            const uint64_t key = wave_nearest_unvisited(g, cx, cy, visited);
            jn = (int32_t)(uint32_t)key;
            dn = (int32_t)(key >> 32);
            slot = kNoSlot;
            prob = -1.0f;
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
                if (prob_out) prob_out[base + lane] = st_prob;
            }
        }
        L += dn;
        c = jn;
    }
    const int64_t s = sq_dist(A.xy[2 * (int64_t)c], A.xy[2 * (int64_t)c + 1],
                              A.xy[2 * (int64_t)start], A.xy[2 * (int64_t)start + 1]);
    L += nint_sqrt(s);
    if (lane == 0) A.lengths[a] = L;
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
    if (lds > 65536)
        ACO_HIP_CHECK(hipFuncSetAttribute((const void *)k_construct,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ConstructArgs A{xy, rows, nnd, grid, n, k, ant0, (uint32_t)iteration, seed,
                    tours, lengths, slots, step_prob};
    k_construct<<<m, kWave, lds, st>>>(A);
    ACO_LAUNCH_CHECK("k_construct");
    return ACO_OK;
}
