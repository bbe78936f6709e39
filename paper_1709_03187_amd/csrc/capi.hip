// Host side of the C ABI: error reporting, device limits and the whole-run
// driver aco_run (set-up, then construction / best tracking / update per
// iteration, all enqueued on the caller's stream).
#include <cmath>
#include <cstdarg>
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>

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

// The error word of each device (word 0; word 1 receives it when taken).
static __device__ __align__(256) uint32_t g_error_word[64];
static std::mutex g_error_mu;
static uint32_t *g_error_ptr[256];

uint32_t *device_error_word()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 256) {
        fail(ACO_ERR_HIP, "no current device for the error word");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_error_mu);
    if (!g_error_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_error_word));
        if (e != hipSuccess || !p) {
            fail(ACO_ERR_HIP, "hipGetSymbolAddress(error word) failed: %s", hipGetErrorString(e));
            return nullptr;
        }
        g_error_ptr[dev] = (uint32_t *)p;
    }
    return g_error_ptr[dev];
}

__global__ void k_take_error(uint32_t *w)
{
    if (threadIdx.x == 0) w[1] = atomicExch(&w[0], 0u);
}

int report_device_error(hipStream_t st)
{
    uint32_t *w = device_error_word();
    if (!w) return ACO_ERR_HIP;
    k_take_error<<<1, 64, 0, st>>>(w);
    ACO_LAUNCH_CHECK("k_take_error");
    uint32_t v = 0;
    ACO_HIP_CHECK(hipMemcpyAsync(&v, w + 1, 4, hipMemcpyDeviceToHost, st));
    ACO_HIP_CHECK(hipStreamSynchronize(st));
    if (v == 0) return ACO_OK;
    static const char *names[] = {
        "construction took a next city out of range",
        "a local best row is not a permutation of 0..n-1",
        "a local best length is not a possible tour length",
        "a tour passed to the pheromone update holds a city out of range",
        "a tour length is <= 0, or m * quantum could overflow int64 (lower deposit_shift)"};
    std::string msg = "device-side check failed:";
    for (int b = 0; b < 5; ++b)
        if (v & (1u << b)) msg += std::string(" [") + names[b] + "]";
    return fail(ACO_ERR_DEVICE, "%s", msg.c_str());
}

int load_params(const aco_params_t *p, aco_params_t &out)
{
    ACO_REQUIRE(p != nullptr, "NULL params");
    const size_t least = offsetof(aco_params_t, seed) + sizeof(p->seed);
    ACO_REQUIRE(p->struct_size >= least, "params struct_size = %u is below %zu", p->struct_size,
                least);
    out = aco_params_t{};
    out.eta_mode = ACO_ETA_DISTANCE;
    out.mlp_w = nullptr;
    std::memcpy(&out, p, std::min((size_t)p->struct_size, sizeof(out)));
    out.struct_size = sizeof(out);
    return ACO_OK;
}

__global__ void k_set_i64(int64_t *p, int64_t v)
{
    if (threadIdx.x == 0) *p = v;
}

// Carves the aco_run workspace into 256-byte aligned arrays (with the learned
// heuristic, also the edge features and their workspace).
struct RunLayout {
    size_t nn, nnd, rev, eta_b, grid, tau, cws, tours, lengths, slots, uws, feat, fws, total;
    size_t grid_bytes, cws_bytes, uws_bytes, fws_bytes;
    RunLayout(int32_t n, int32_t k, int32_t m, bool learned = false)
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
        fws_bytes = learned ? aco_features_workspace_bytes() : 0;
        feat = o;    o = al(o + (learned ? nk * 32 : 0));
        fws = o;     o = al(o + fws_bytes);
        total = o;
    }
};

static int validate_params(int32_t n, const aco_params_t *p)
{
    ACO_REQUIRE(p != nullptr, "NULL params");
    ACO_REQUIRE(p->eta_mode == ACO_ETA_DISTANCE || p->eta_mode == ACO_ETA_LEARNED,
                "eta_mode = %d unknown", p->eta_mode);
    ACO_REQUIRE(p->eta_mode != ACO_ETA_LEARNED || p->mlp_w, "ACO_ETA_LEARNED needs mlp_w");
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
    case ACO_ERR_DEVICE: return "ACO_ERR_DEVICE";
    default: return "ACO_ERR_UNKNOWN";
    }
}

extern "C" const char *aco_last_error(void) { return g_last_error; }

extern "C" int aco_device_error(void *stream)
{
    clear_error();
    return report_device_error(as_stream(stream));
}

extern "C" const char *aco_version(void) { return "aco-mi355x 0.1 (gfx950)"; }

extern "C" size_t aco_workspace_bytes(int32_t which, int32_t n, int32_t k, int32_t m)
{
    switch (which) {
    case ACO_WS_GRID: return aco_grid_bytes(n);
    case ACO_WS_CONSTRUCT: return aco_construct_workspace_bytes(n, k);
    case ACO_WS_UPDATE: return aco_update_workspace_bytes(n, k, m);
    case ACO_WS_RUN: {
        aco_params_t q{};
        q.struct_size = sizeof(q);
        q.m = m;
        q.k = k;
        return aco_run_workspace_bytes(n, &q);
    }
    case ACO_WS_TWO_OPT: return aco_two_opt_workspace_bytes(n, m, 1);
    case ACO_WS_FEATURES: return aco_features_workspace_bytes();
    case ACO_WS_MLP_BACKWARD:
        return (n < 1 || k < 1) ? 0 : aco_mlp_backward_workspace_bytes((int64_t)n * k);
    default: return 0;
    }
}

extern "C" size_t aco_run_workspace_bytes(int32_t n, const aco_params_t *pin)
{
    aco_params_t q;
    if (load_params(pin, q) != ACO_OK || n < 3 || q.k < 1 || q.m < 1) return 0;
    return RunLayout(n, q.k, q.m, q.eta_mode == ACO_ETA_LEARNED).total;
}

extern "C" int aco_run(const int32_t *xy, int32_t n, const aco_params_t *pin, int32_t *best_tour,
                       int64_t *best_len, int64_t *iter_best, float *tau_out, void *ws,
                       size_t ws_bytes, void *stream)
{
    clear_error();
    aco_params_t q;
    int rc = load_params(pin, q);
    if (rc != ACO_OK) return rc;
    const aco_params_t *p = &q;
    rc = validate_params(n, p);
    if (rc != ACO_OK) return rc;
    ACO_REQUIRE(xy && best_tour && best_len && ws, "NULL array argument");
    const int32_t k = p->k, m = p->m;
    const bool learned = p->eta_mode == ACO_ETA_LEARNED;
    const RunLayout lay(n, k, m, learned);
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
    if (learned) {   // eta_b = sigmoid(network score)^beta
        float *feat = (float *)(b + lay.feat);
        rc = aco_edge_features(xy, n, k, nn, nnd, rev, feat, b + lay.fws, lay.fws_bytes, stream);
        if (rc != ACO_OK) return rc;
        rc = aco_mlp_forward(feat, (int64_t)n * k, p->mlp_w, ACO_MLP_OUT_ETA_B, p->beta, eta_b,
                             stream);
        if (rc != ACO_OK) return rc;
    }
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
