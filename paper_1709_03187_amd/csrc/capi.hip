// Host side of the C ABI: error reporting, device limits and the whole-run
// driver aco_run (set-up, then construction / best tracking / update per
// iteration, all enqueued on the caller's stream).
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "common.hpp"
#include "device.hpp"

namespace aco {

static thread_local char g_last_error[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_last_error[0] = '\0'; }

int num_cus()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1;
    return v > 0 ? v : 1;
}

size_t max_lds_per_block()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    return v > 0 ? (size_t)v : 65536;
}

__global__ void k_set_i64(int64_t *p, int64_t v)
{
    if (threadIdx.x == 0) *p = v;
}

// Carves the aco_run workspace into 256-byte aligned arrays.
struct RunLayout {
    size_t nn, nnd, rev, eta_b, grid, tau, cws, tours, lengths, slots, uws, total;
    size_t grid_bytes, cws_bytes, uws_bytes;
    RunLayout(int32_t n, int32_t k, int32_t m)
    {
        auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
        const size_t nk = (size_t)n * k, mn = (size_t)m * n;
        grid_bytes = aco_grid_bytes(n);
        cws_bytes = aco_construct_workspace_bytes(n, k);
        uws_bytes = aco_update_workspace_bytes(n, k, m);
        size_t o = 0;
        nn = o;      o = al(o + nk * 4);
        nnd = o;     o = al(o + nk * 4);
        rev = o;     o = al(o + nk);
        eta_b = o;   o = al(o + nk * 4);
        grid = o;    o = al(o + grid_bytes);
        tau = o;     o = al(o + nk * 4);
        cws = o;     o = al(o + cws_bytes);
        tours = o;   o = al(o + mn * 4);
        lengths = o; o = al(o + (size_t)m * 8);
        slots = o;   o = al(o + mn);
        uws = o;     o = al(o + uws_bytes);
        total = o;
    }
};

static int validate_params(int32_t n, const aco_params_t *p)
{
    ACO_REQUIRE(p != nullptr, "NULL params");
    ACO_REQUIRE(n >= 3 && n <= (1 << 27), "n = %d out of range [3, 2^27]", n);
    ACO_REQUIRE(p->k >= 1 && p->k <= ACO_MAX_K && p->k <= n - 1, "k = %d out of range", p->k);
    ACO_REQUIRE(p->m >= 1 && p->m <= (1 << 20), "m = %d out of range [1, 2^20]", p->m);
    ACO_REQUIRE(std::isfinite(p->alpha) && p->alpha >= 0, "alpha must be finite and >= 0");
    ACO_REQUIRE(std::isfinite(p->beta) && p->beta >= 0, "beta must be finite and >= 0");
    ACO_REQUIRE(p->rho > 0.0 && p->rho <= 1.0, "rho must lie in (0, 1]");
    ACO_REQUIRE(p->iterations >= 0, "iterations must be >= 0");
    ACO_REQUIRE(p->deposit_shift >= 0 && p->deposit_shift <= 62, "deposit_shift out of [0, 62]");
    return ACO_OK;
}

}  // namespace aco

using namespace aco;

extern "C" const char *aco_strerror(int code)
{
    switch (code) {
    case ACO_OK: return "ACO_OK";
    case ACO_ERR_INVALID_ARG: return "ACO_ERR_INVALID_ARG";
    case ACO_ERR_UNSUPPORTED: return "ACO_ERR_UNSUPPORTED";
    case ACO_ERR_DEGENERATE: return "ACO_ERR_DEGENERATE";
    case ACO_ERR_WORKSPACE: return "ACO_ERR_WORKSPACE";
    case ACO_ERR_HIP: return "ACO_ERR_HIP";
    default: return "ACO_ERR_UNKNOWN";
    }
}

extern "C" const char *aco_last_error(void) { return g_last_error; }

extern "C" const char *aco_version(void) { return "aco-mi355x 0.1 (gfx950)"; }

extern "C" size_t aco_run_workspace_bytes(int32_t n, const aco_params_t *p)
{
    if (!p || n < 3 || p->k < 1 || p->m < 1) return 0;
    return RunLayout(n, p->k, p->m).total;
}

extern "C" int aco_run(const int32_t *xy, int32_t n, const aco_params_t *p, int32_t *best_tour,
                       int64_t *best_len, int64_t *iter_best, float *tau_out, void *ws,
                       size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = validate_params(n, p);
    if (rc != ACO_OK) return rc;
    ACO_REQUIRE(xy && best_tour && best_len && ws, "NULL array argument");
    const int32_t k = p->k, m = p->m;
    const RunLayout lay(n, k, m);
    if (ws_bytes < lay.total)
        return fail(ACO_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total);
    hipStream_t st = as_stream(stream);
    char *b = (char *)ws;
    int32_t *nn = (int32_t *)(b + lay.nn);
    int32_t *nnd = (int32_t *)(b + lay.nnd);
    int8_t *rev = (int8_t *)(b + lay.rev);
    float *eta_b = (float *)(b + lay.eta_b);
    void *grid = b + lay.grid;
    float *tau = (float *)(b + lay.tau);
    int32_t *tours = (int32_t *)(b + lay.tours);
    int64_t *lengths = (int64_t *)(b + lay.lengths);
    uint8_t *slots = (uint8_t *)(b + lay.slots);

    rc = aco_build_candidates(xy, n, k, p->beta, nullptr, nn, nnd, rev, eta_b, grid,
                              lay.grid_bytes, stream);
    if (rc != ACO_OK) return rc;
    int64_t L_nn = 0;
    rc = aco_init_pheromone(xy, n, k, nn, nnd, grid, best_tour, tau, nullptr, &L_nn, stream);
    if (rc != ACO_OK) return rc;
    k_set_i64<<<1, 64, 0, st>>>(best_len, L_nn);
    ACO_LAUNCH_CHECK("k_set_i64");
    for (int32_t it = 0; it < p->iterations; ++it) {
        rc = aco_construct_tours(xy, n, k, nn, nnd, eta_b, grid, tau, m, 0, p->alpha, p->seed, it,
                                 tours, lengths, slots, nullptr, b + lay.cws, lay.cws_bytes,
                                 stream);
        if (rc != ACO_OK) return rc;
        rc = aco_track_best(n, m, tours, lengths, best_len, best_tour,
                            iter_best ? iter_best + it : nullptr, stream);
        if (rc != ACO_OK) return rc;
        rc = aco_update_pheromone(n, k, nn, rev, m, tours, slots, lengths, p->rho,
                                  p->deposit_shift, tau, b + lay.uws, lay.uws_bytes, stream);
        if (rc != ACO_OK) return rc;
    }
    if (tau_out)
        ACO_HIP_CHECK(hipMemcpyAsync(tau_out, tau, (size_t)n * k * 4, hipMemcpyDeviceToDevice, st));
    return ACO_OK;
}
