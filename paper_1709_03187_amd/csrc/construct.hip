// Tour construction with the random proportional rule (Section 2, Eq. 1), one
// instance.
//
// One ant per 64-wide wavefront, cities named by their position in the grid's
// cell order.  Per step the ant at city c reads the packed candidate row
// {nn[c][r], w[c][r]} (one 128-byte line at k = 16), tests the
// candidates against its visited bitmask in LDS, forms the FP64 running sum of
// the unvisited weights across lanes, and picks the first lane whose running
// sum exceeds u * S with a ballot.  When no unvisited candidate has positive
// weight the wave takes the nearest unvisited city (256-NN table, then grid).
// The tour's length is summed exactly inside the same kernel.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>

#include "colony.hpp"
#include "common.hpp"

namespace aco {

// Choice weights of every row, by position in cell order: the row of city i
// is row pinv[i] of the table, its candidates named by position (the first k
// entries of the grid's neighbour table by position, the same (d, index)-
// ordered list the candidate list is a prefix of).  One lane per element, an
// aligned group of KP lanes per row, rows in city order: tau and eta_b are
// read as streams, each row's candidates as one contiguous read, and each
// row is written whole by its group (one 128-byte line at k = 16).
template <int KP>
__global__ __launch_bounds__(256) void k_choice_info(const int32_t *__restrict__ pinv,
                                                     const int32_t *__restrict__ ext_pos,
                                                     int32_t kxp, const float *__restrict__ tau,
                                                     const float *__restrict__ eta_b, int32_t n,
                                                     int32_t k, double alpha,
                                                     CandW *__restrict__ rows)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t i = t / KP;
    const int r = (int)(t % KP);
    const bool act = i < n && r < k;
    int64_t q = 0;
    int32_t pos = 0;
    float tv = 0.0f, ev = 0.0f;
    if (act) {
        q = pinv[i];
        pos = ext_pos[q * kxp + r];
        tv = tau[i * k + r];
        ev = eta_b[i * k + r];
    }
    const float w = choice_weight_lane<KP>(act, tv, ev, alpha);   // every lane takes part
    if (act) rows[q * row_stride(KP) + r] = CandW{pos, w};
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
    const int32_t *lbest;   // [m][n] local best tours (PartialACO) or nullptr
    const int64_t *lbest_len;   // [m] their exact lengths, or nullptr
    uint64_t p_threshold;
    int32_t max_modify;
    int32_t m;              // ants in this launch
    int32_t ant_lds;        // LDS bytes per ant (visited set, Independent Roulette's uniforms)
    uint32_t *err;          // the device's error word
    uint64_t *prof;         // step profile build: [m][kProfFields] counters, else nullptr
};

// One ant per wave, up to four waves (ants) per workgroup, each with its own
// slice of the workgroup's LDS (the visited bitmask).  A workgroup's waves go
// to different SIMDs of its CU, so with one workgroup per CU no two ants share
// a SIMD (as separate one-wave workgroups, about a fifth of the ants did, and
// ran about 5% slower on average, up to 12% for the slowest).
// kSampler: 0 the roulette of Eq. 1, 1 Independent Roulette; kProb: the step
// probabilities are recorded (one variant per kernel keeps the step lean).
template <int KP, int kSampler, bool kProb>
__global__ __launch_bounds__(4 * kWave) void k_construct(ConstructArgs A)
{
    extern __shared__ uint32_t lds[];
    // the wave's index, stated uniform (the compiler would otherwise treat
    // everything derived from it, the ant's pointers and loop bounds, as per lane)
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int32_t a = (int32_t)blockIdx.x * (int32_t)(blockDim.x / kWave) + wave;   // ant
    if (a >= A.m) return;                          // (no barriers in this kernel)
    uint32_t *vis = lds + (size_t)wave * (size_t)A.ant_lds / 4;
    AntTask T;
    T.xy = A.xy;
    T.rows = A.rows;
    T.n = A.n;
    T.k = A.k;
    T.ant = (uint32_t)(A.ant0 + a);               // absolute ant index (Philox counter)
    T.iteration = A.iteration;
    T.seed = A.seed;
    T.tour = A.tours + (int64_t)a * A.n;
    T.slots = A.slots + (int64_t)a * A.n;
    T.prob = A.step_prob ? A.step_prob + (int64_t)a * A.n : nullptr;
    T.lbest = A.lbest ? A.lbest + (int64_t)a * A.n : nullptr;
    T.lbest_len = A.lbest && A.lbest_len ? A.lbest_len + a : nullptr;
    T.p_threshold = A.p_threshold;
    T.max_modify = A.max_modify;
    T.err = A.err;
    T.prof = A.prof ? A.prof + (int64_t)a * kProfFields : nullptr;
    if constexpr (kSampler != 0)   // the uniforms follow the visited set, 16-byte aligned
        T.ir_words = vis + ((((int64_t)A.n + 31) / 32 * 4 + 15) & ~(int64_t)15) / 4;
    const int64_t len = build_ant_fixed<KP, kProb, PositionSpace, kSampler, true>(
        T, VisBits{vis}, [&]() { return grid_view(A.grid); });
    if (lane_id() == 0) A.lengths[a] = len;     // exact closed length
}

}  // namespace aco

using namespace aco;

// Where the step profile build writes its counters (set by
// aco_step_profile_buffer; always null in the library itself).
static uint64_t *g_step_profile = nullptr;

#ifdef ACO_STEP_PROFILE
// Step profile build only: the device buffer ([m][16] uint64) that the next
// constructions fill with each ant's clock counters (NULL to stop).
extern "C" void aco_step_profile_buffer(uint64_t *buf) { g_step_profile = buf; }
// The grid-search counters of this library's construction kernels: copied to
// host[4] (searches, passes, batches of 64 points, points in the searched
// ranges), zeroed, and counting switched on (on != 0) or off for the launches
// that follow.
extern "C" int aco_grid_stats(uint64_t *host, int on)
{
    unsigned long long zero[4] = {0, 0, 0, 0};
    if (hipMemcpyFromSymbol(host, HIP_SYMBOL(g_grid_stats), sizeof(zero)) != hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(g_grid_stats), zero, sizeof(zero)) != hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(g_grid_on), &on, sizeof(on)) != hipSuccess)
        return ACO_ERR_HIP;
    return ACO_OK;
}
#endif

extern "C" size_t aco_construct_workspace_bytes(int32_t n, int32_t k)
{
    if (n < 1 || k < 1) return 0;
    return (size_t)n * (size_t)row_stride(k) * sizeof(CandW);
}

static int construct(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                     const int32_t *nnd, const float *eta_b, const void *grid, const float *tau,
                     int32_t m, int32_t ant0, double alpha, uint64_t seed, int64_t iteration,
                     const int32_t *lbest, const int64_t *lbest_len, uint64_t p_threshold,
                     int32_t max_modify, int32_t sampler, int32_t *tours, int64_t *lengths,
                     uint8_t *slots, float *step_prob, void *ws, size_t ws_bytes, void *stream)
{
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
    size_t lds = bitmask_bytes(n);
    if (sampler == ACO_SAMPLER_INDEPENDENT)   // plus one block of uniforms (64 steps)
        lds = ((lds + 15) & ~(size_t)15) + (size_t)kWave * ir_words_per_step(k) * 4;
    lds = (lds + 15) & ~(size_t)15;            // one ant's slice
    if (lds > max_lds_per_block())
        return fail(ACO_ERR_UNSUPPORTED, "visited set (and uniforms) of %zu bytes exceed LDS (%zu)",
                    lds, max_lds_per_block());
    hipStream_t st = as_stream(stream);
    CandW *rows = (CandW *)ws;
    const GridLayout lay(n);
    const int32_t *pinv = (const int32_t *)((const char *)grid + lay.pinv);
    const int32_t *ext_pos = (const int32_t *)((const char *)grid + lay.ext_pos);
    {
        const int kp = k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64;
        auto ci = k <= 8 ? k_choice_info<8> : k <= 16 ? k_choice_info<16>
                : k <= 32 ? k_choice_info<32> : k_choice_info<64>;
        ci<<<blocks_for((int64_t)n * kp, 256), 256, 0, st>>>(pinv, ext_pos, ext_pos_width(n), tau,
                                                              eta_b, n, k, alpha, rows);
        ACO_LAUNCH_CHECK("k_choice_info");
    }
    void (*kern)(ConstructArgs);
    if (sampler == ACO_SAMPLER_INDEPENDENT)   // no step probabilities (checked above)
        kern = k <= 8 ? k_construct<8, 1, false> : k <= 16 ? k_construct<16, 1, false>
             : k <= 32 ? k_construct<32, 1, false> : k_construct<64, 1, false>;
    else if (step_prob)
        kern = k <= 8 ? k_construct<8, 0, true> : k <= 16 ? k_construct<16, 0, true>
             : k <= 32 ? k_construct<32, 0, true> : k_construct<64, 0, true>;
    else
        kern = k <= 8 ? k_construct<8, 0, false> : k <= 16 ? k_construct<16, 0, false>
             : k <= 32 ? k_construct<32, 0, false> : k_construct<64, 0, false>;
    // up to four ants per CU (one per SIMD): one workgroup of four ants per CU,
    // the LDS request padded past half the CU's so that no CU takes two; more
    // ants than that (or slices too large for four): one ant per workgroup, as
    // many resident as the LDS allows
    const size_t lmax = max_lds_per_block();
    const int wpb = ((int64_t)m <= 4 * (int64_t)num_cus() && 4 * lds <= lmax) ? 4 : 1;
    const int32_t blocks = (m + wpb - 1) / wpb;
    size_t lds_req = (size_t)wpb * lds;
    if (wpb == 4 && lds_req <= lmax / 2) lds_req = lmax / 2 + 16;
    if (lds_req > 65536)
        ACO_HIP_CHECK(hipFuncSetAttribute((const void *)kern,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds_req));
    uint32_t *err = device_error_word();
    if (!err) return ACO_ERR_HIP;
    ConstructArgs A{xy,    rows,    grid,      n,     k,           ant0,
                    (uint32_t)iteration,       seed,      tours, lengths, slots,
                    step_prob, lbest,   lbest_len, p_threshold, max_modify, m, (int32_t)lds,
                    err, g_step_profile};
    kern<<<blocks, wpb * kWave, lds_req, st>>>(A);
    ACO_LAUNCH_CHECK("k_construct");
    return ACO_OK;
}

extern "C" int aco_construct_tours(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                                   const int32_t *nnd, const float *eta_b, const void *grid,
                                   const float *tau, int32_t m, int32_t ant0, double alpha,
                                   uint64_t seed, int64_t iteration, int32_t *tours,
                                   int64_t *lengths, uint8_t *slots, float *step_prob, void *ws,
                                   size_t ws_bytes, void *stream)
{
    clear_error();
    return construct(xy, n, k, nn, nnd, eta_b, grid, tau, m, ant0, alpha, seed, iteration,
                     nullptr, nullptr, 0, 0, ACO_SAMPLER_ROULETTE, tours, lengths, slots,
                     step_prob, ws, ws_bytes, stream);
}

extern "C" int aco_construct_partial(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                                     const int32_t *nnd, const float *eta_b, const void *grid,
                                     const float *tau, int32_t m, int32_t ant0, double alpha,
                                     uint64_t seed, int64_t iteration, double p_partial,
                                     int32_t max_modify, const int32_t *lbest, int32_t *tours,
                                     int64_t *lengths, uint8_t *slots, float *step_prob,
                                     void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    ACO_REQUIRE(lbest, "lbest is NULL");
    ACO_REQUIRE(std::isfinite(p_partial) && p_partial >= 0.0 && p_partial <= 1.0,
                "p_partial = %g out of [0, 1]", p_partial);
    ACO_REQUIRE(max_modify >= 1, "max_modify = %d must be >= 1", max_modify);
    // P = round(p 2^32), ties to even (the current rounding mode)
    const uint64_t thr = (uint64_t)std::nearbyint(std::ldexp(p_partial, 32));
    return construct(xy, n, k, nn, nnd, eta_b, grid, tau, m, ant0, alpha, seed, iteration, lbest,
                     nullptr, thr, max_modify, ACO_SAMPLER_ROULETTE, tours, lengths, slots,
                     step_prob, ws, ws_bytes, stream);
}

extern "C" int aco_construct_ex(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                                const int32_t *nnd, const float *eta_b, const void *grid,
                                const float *tau, int32_t m, int32_t ant0, double alpha,
                                uint64_t seed, int64_t iteration, const aco_construct_opts_t *opts,
                                int32_t *tours, int64_t *lengths, uint8_t *slots,
                                float *step_prob, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    aco_construct_opts_t o{sizeof(aco_construct_opts_t), ACO_SAMPLER_ROULETTE, 0.0, 0, nullptr,
                           nullptr};
    if (opts) {
        const size_t least = offsetof(aco_construct_opts_t, lbest) + sizeof(o.lbest);
        ACO_REQUIRE(opts->struct_size >= least, "opts->struct_size = %u is below %zu",
                    opts->struct_size, least);
        std::memcpy(&o, opts, std::min((size_t)opts->struct_size, sizeof(o)));
    }
    ACO_REQUIRE(o.sampler == ACO_SAMPLER_ROULETTE || o.sampler == ACO_SAMPLER_INDEPENDENT,
                "sampler = %d unknown", o.sampler);
    ACO_REQUIRE(o.sampler == ACO_SAMPLER_ROULETTE || !step_prob,
                "step_prob is only defined for the roulette sampler");
    uint64_t thr = 0;
    if (o.lbest) {
        ACO_REQUIRE(std::isfinite(o.p_partial) && o.p_partial >= 0.0 && o.p_partial <= 1.0,
                    "p_partial = %g out of [0, 1]", o.p_partial);
        ACO_REQUIRE(o.max_modify >= 1, "max_modify = %d must be >= 1", o.max_modify);
        thr = (uint64_t)std::nearbyint(std::ldexp(o.p_partial, 32));
    }
    return construct(xy, n, k, nn, nnd, eta_b, grid, tau, m, ant0, alpha, seed, iteration,
                     o.lbest, o.lbest_len, thr, o.max_modify, o.sampler, tours, lengths, slots,
                     step_prob, ws, ws_bytes, stream);
}
