// Pheromone update (Section 2, Eq. 2-4) and best-tour tracking.
//
// Deposits are accumulated in int64 fixed point (q_a = floor(2^shift / L_a)
// per ant, i.e. 1/C^a with `shift` fraction bits) by integer atomics, so the
// sum is independent of the order in which ants and edges arrive; the merge
// then applies evaporation and the deposit with exactly two FP32 roundings.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "device.hpp"

namespace aco {

// q_a = floor(2^shift / L_a).  Every slot's sum stays below m * max q_a, so
// m * q_a < 2^63 for every ant keeps the int64 sums exact; otherwise (or for
// a length <= 0, whose quantum is set to 0) a guard trips.
__global__ void k_quanta(const int64_t *__restrict__ lengths, int32_t m, int32_t shift,
                         int64_t *__restrict__ q, uint32_t *err)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= m) return;
    const int64_t L = lengths[a];
    const int64_t qa = L > 0 ? ((int64_t)1 << shift) / L : 0;
    if (L <= 0 || qa > INT64_MAX / m) flag_error(err, kErrLength);
    q[a] = qa;
}

__global__ void k_zero_i64(int64_t *p, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__device__ __forceinline__ int find_slot(const int32_t *__restrict__ nn, int64_t row, int k,
                                         int32_t city)
{
    for (int r = 0; r < k; ++r)
        if (nn[row + r] == city) return r;
    return -1;
}

// One thread per tour edge (tour[t], tour[t+1 mod n]): ant a = blockIdx.y
// (a 2-D grid, so no index division).  The slot of the forward direction
// comes from the construction record when it names the edge; the reverse
// slot from rev[] or, for edges outside the forward list, a scan of the other
// row.
__global__ void k_deposit(const int32_t *__restrict__ nn, const int8_t *__restrict__ rev,
                          int32_t n, int32_t k, int32_t a0, const int32_t *__restrict__ tours,
                          const uint8_t *__restrict__ slots, const int64_t *__restrict__ q,
                          unsigned long long *__restrict__ acc, uint32_t *err)
{
    const int32_t a = a0 + (int32_t)blockIdx.y;
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t base = (int64_t)a * n;
    const int32_t i = tours[base + t];
    const int32_t j = tours[base + (t + 1 == n ? 0 : t + 1)];
    // not a tour of 0..n-1: nothing deposited for the edge, reported once per wave
    const bool bad = i < 0 || i >= n || j < 0 || j >= n;
    if (__builtin_amdgcn_ballot_w64(bad) != 0ull && lane_id() == 0) flag_error(err, kErrTourCity);
    if (bad) return;
    const unsigned long long qa = (unsigned long long)q[a];
    const int64_t ri = (int64_t)i * k, rj = (int64_t)j * k;
    // A fallback move (slot 255) can still end on a candidate city: that happens
    // when every unvisited candidate has zero weight.  Such edges are located
    // by scanning the row, as are edges without a construction record.
    int r = -1;
    if (slots && t + 1 < n) {   // the record is trusted (checking it costs a gather)
        const uint32_t s = slots[base + t + 1];
        if (s < (uint32_t)k) r = (int)s;
    }
    if (r < 0) r = find_slot(nn, ri, k, j);
    const int r2 = (r >= 0) ? (int)rev[ri + r] : find_slot(nn, rj, k, i);
    // one atomic per undirected edge, into its canonical slot: the slot in the
    // row of the smaller city when both directions are stored (one atomic
    // instruction for both cases)
    const int64_t dst = (r >= 0 && (r2 < 0 || i < j)) ? ri + r
                        : (r2 >= 0 && r2 < k)          ? rj + r2
                                                        : -1;
    if (dst >= 0) atomicAdd(&acc[dst], qa);
}

// tau = fl32(fl32(tau * f) + fl32(fl32(acc) * 2^-shift)); both products are
// exact or singly rounded, no fused multiply-add.  The deposit of slot (i, r)
// sits in the canonical slot of its edge: its own, or the partner slot
// (nn[i][r], rev[i][r]) when that one lies in the row of the smaller city.
__global__ void k_merge(float *__restrict__ tau, const int64_t *__restrict__ acc,
                        const int32_t *__restrict__ nn, const int8_t *__restrict__ rev,
                        int32_t k, int64_t count, float f, float scale)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = (count <= INT32_MAX) ? (int64_t)((uint32_t)e / (uint32_t)k) : e / k;
        const int32_t j = nn[e];
        const int r2 = rev[e];
        const int64_t src = (r2 >= 0 && j < i) ? (int64_t)j * k + r2 : e;
        const float evap = __fmul_rn(tau[e], f);
        const float dep = __fmul_rn((float)acc[src], scale);
        tau[e] = __fadd_rn(evap, dep);
    }
}

// ---------------------------------------------------------------- best tour

__device__ __forceinline__ int64_t wave_min_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

// Block-wide minimum (blockDim.x a multiple of 64, at most 1024).
__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t *red)
{
    v = wave_min_i64(v);
    if (lane_id() == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    int64_t r = INT64_MAX;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) r = red[w] < r ? red[w] : r;
    __syncthreads();
    return r;
}

// Iteration best: the smallest length, lowest ant on ties.
__device__ __forceinline__ int32_t best_ant(const int64_t *lengths, int32_t m)
{
    __shared__ int64_t red[1024 / kWave];
    int64_t lmin = INT64_MAX;
    for (int a = threadIdx.x; a < m; a += blockDim.x) lmin = lengths[a] < lmin ? lengths[a] : lmin;
    lmin = block_min_i64(lmin, red);
    int64_t amin = INT64_MAX;
    for (int a = threadIdx.x; a < m; a += blockDim.x)
        if (lengths[a] == lmin && a < amin) amin = a;
    return (int32_t)block_min_i64(amin, red);
}

// Every block finds the iteration best and copies its share of that tour if
// it beats the best so far (best_len is only read here).
__global__ __launch_bounds__(256) void k_best_copy(const int32_t *__restrict__ tours,
                                                   const int64_t *__restrict__ lengths, int32_t n,
                                                   int32_t m, const int64_t *best_len,
                                                   int32_t *best_tour)
{
    const int32_t a = best_ant(lengths, m);
    if (lengths[a] >= *best_len) return;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        best_tour[t] = tours[(int64_t)a * n + t];
}

__global__ __launch_bounds__(256) void k_best_finish(const int64_t *__restrict__ lengths,
                                                     int32_t m, int64_t *best_len,
                                                     int64_t *iter_best)
{
    const int32_t a = best_ant(lengths, m);
    if (threadIdx.x == 0) {
        const int64_t L = lengths[a];
        if (iter_best) *iter_best = L;
        if (L < *best_len) *best_len = L;
    }
}

// Pheromone from the local best tours (the P-ACO variant of Section 3): the
// quantum of local best a is q_a = floor(2^shift * L_g / L_a) with the ratio
// in FP64 and L_g the shortest local best (one workgroup).
// A length <= 0 trips a guard and gets quantum 0.
__global__ __launch_bounds__(1024) void k_quanta_ratio(const int64_t *__restrict__ lbest_len,
                                                       int32_t m, int32_t shift,
                                                       int64_t *__restrict__ q, uint32_t *err)
{
    __shared__ int64_t red[1024 / kWave];
    int64_t lmin = INT64_MAX;
    for (int a = threadIdx.x; a < m; a += blockDim.x)
        if (lbest_len[a] > 0) lmin = lbest_len[a] < lmin ? lbest_len[a] : lmin;
    const int64_t Lg = block_min_i64(lmin, red);
    for (int a = threadIdx.x; a < m; a += blockDim.x) {
        const int64_t L = lbest_len[a];
        if (L <= 0) flag_error(err, kErrLength);
        q[a] = L > 0 ? (int64_t)floor(ldexp((double)Lg / (double)L, shift)) : 0;
    }
}

// tau = fl32(base + fl32(fl32(acc) * scale)), no evaporation; the canonical
// slot rule as in k_merge.
__global__ void k_merge_base(float *__restrict__ tau, const int64_t *__restrict__ acc,
                             const int32_t *__restrict__ nn, const int8_t *__restrict__ rev,
                             int32_t k, int64_t count, float base, float scale)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = (count <= INT32_MAX) ? (int64_t)((uint32_t)e / (uint32_t)k) : e / k;
        const int32_t j = nn[e];
        const int r2 = rev[e];
        const int64_t src = (r2 >= 0 && j < i) ? (int64_t)j * k + r2 : e;
        tau[e] = __fadd_rn(base, __fmul_rn((float)acc[src], scale));
    }
}

// PartialACO local bests (Algorithm 1): ant a's row is replaced when its new
// tour is strictly shorter.  The copy reads lbest_len, the second kernel then
// updates it, so every block of the copy sees the old value.
__global__ void k_lbest_copy(const int32_t *__restrict__ tours, const int64_t *__restrict__ lengths,
                             int32_t n, int32_t a0, const int64_t *__restrict__ lbest_len,
                             int32_t *__restrict__ lbest)
{
    const int32_t a = a0 + (int32_t)blockIdx.y;
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n || lengths[a] >= lbest_len[a]) return;
    lbest[(int64_t)a * n + t] = tours[(int64_t)a * n + t];
}

__global__ void k_lbest_len(const int64_t *__restrict__ lengths, int32_t m, int64_t *lbest_len)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < m && lengths[a] < lbest_len[a]) lbest_len[a] = lengths[a];
}

}  // namespace aco

using namespace aco;

extern "C" size_t aco_update_workspace_bytes(int32_t n, int32_t k, int32_t m)
{
    if (n < 1 || k < 1 || m < 1) return 0;
    return (size_t)n * (size_t)k * 8 + (((size_t)m * 8 + 255) & ~(size_t)255);
}

static int validate_update(int32_t n, int32_t k, const int32_t *nn, const int8_t *rev, int32_t m,
                           const int32_t *tours, const int64_t *lengths, double rho,
                           int32_t deposit_shift, const float *tau)
{
    ACO_REQUIRE(n >= 3 && n <= (1 << 27), "n = %d out of range [3, 2^27]", n);
    ACO_REQUIRE(k >= 1 && k <= ACO_MAX_K && k <= n - 1, "k = %d out of range", k);
    ACO_REQUIRE(m >= 1 && m <= (1 << 20), "m = %d out of range [1, 2^20]", m);
    ACO_REQUIRE(rho > 0.0 && rho <= 1.0, "rho must lie in (0, 1]");
    ACO_REQUIRE(deposit_shift >= 0 && deposit_shift <= 62, "deposit_shift out of [0, 62]");
    ACO_REQUIRE(nn && rev && tours && lengths && tau, "NULL array argument");
    return ACO_OK;
}

// Evaporation and deposit with the slot sums and quanta in `ws` (validated).
static int update_pheromone(int32_t n, int32_t k, const int32_t *nn, const int8_t *rev, int32_t m,
                            const int32_t *tours, const uint8_t *slots, const int64_t *lengths,
                            double rho, int32_t deposit_shift, float *tau, void *ws,
                            hipStream_t st)
{
    const int64_t nk = (int64_t)n * k;
    int64_t *acc = (int64_t *)ws;
    int64_t *q = (int64_t *)((char *)ws + (size_t)nk * 8);
    uint32_t *err = device_error_word();
    if (!err) return ACO_ERR_HIP;
    k_zero_i64<<<std::min(4096u, blocks_for(nk, 256)), 256, 0, st>>>(acc, nk);
    k_quanta<<<blocks_for(m, 256), 256, 0, st>>>(lengths, m, deposit_shift, q, err);
    for (int32_t a0 = 0; a0 < m; a0 += 65535) {   // grid y is at most 65,535 ants
        const int32_t ma = m - a0 < 65535 ? m - a0 : 65535;
        k_deposit<<<dim3(blocks_for(n, 256), (unsigned)ma), 256, 0, st>>>(
            nn, rev, n, k, a0, tours, slots, q, (unsigned long long *)acc, err);
    }
    const float f = (float)(1.0 - rho);
    const float scale = std::ldexp(1.0f, -deposit_shift);
    k_merge<<<std::min(8192u, blocks_for(nk, 256)), 256, 0, st>>>(tau, acc, nn, rev, k, nk, f,
                                                                  scale);
    ACO_LAUNCH_CHECK("update kernels");
    return ACO_OK;
}

extern "C" int aco_update_pheromone(int32_t n, int32_t k, const int32_t *nn, const int8_t *rev,
                                    int32_t m, const int32_t *tours, const uint8_t *slots,
                                    const int64_t *lengths, double rho, int32_t deposit_shift,
                                    float *tau, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = validate_update(n, k, nn, rev, m, tours, lengths, rho, deposit_shift, tau);
    if (rc != ACO_OK) return rc;
    ACO_REQUIRE(ws, "NULL workspace");
    const size_t need = aco_update_workspace_bytes(n, k, m);
    if (ws_bytes < need)
        return fail(ACO_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    return update_pheromone(n, k, nn, rev, m, tours, slots, lengths, rho, deposit_shift, tau, ws,
                            as_stream(stream));
}

// The update's scratch for callers that cannot allocate: the slot sums and
// quanta of one update, held by the library on every device it runs on.
// Host code uses only the device address taken below, never this name.
static __device__ __align__(256) unsigned char scratch[ACO_UPDATE_STATIC_BYTES];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[256];

// Device address of this device's scratch, located on the first call per device.
static int scratch_address(void **out)
{
    int dev = 0;
    ACO_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 256) return fail(ACO_ERR_HIP, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        ACO_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(ACO_ERR_HIP, "no device address for the update scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ACO_OK;
}

extern "C" int aco_update_pheromone_static(int32_t n, int32_t k, const int32_t *nn,
                                           const int8_t *rev, int32_t m, const int32_t *tours,
                                           const uint8_t *slots, const int64_t *lengths,
                                           double rho, int32_t deposit_shift, float *tau,
                                           void *stream)
{
    clear_error();
    int rc = validate_update(n, k, nn, rev, m, tours, lengths, rho, deposit_shift, tau);
    if (rc != ACO_OK) return rc;
    const size_t need = aco_update_workspace_bytes(n, k, m);
    ACO_REQUIRE(need <= (size_t)ACO_UPDATE_STATIC_BYTES,
                "n k 8 + m 8 = %zu bytes exceed the %u bytes of the static scratch", need,
                (unsigned)ACO_UPDATE_STATIC_BYTES);
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != ACO_OK) return rc;
    return update_pheromone(n, k, nn, rev, m, tours, slots, lengths, rho, deposit_shift, tau, ws,
                            as_stream(stream));
}

extern "C" int aco_track_best(int32_t n, int32_t m, const int32_t *tours, const int64_t *lengths,
                              int64_t *best_len, int32_t *best_tour, int64_t *iter_best,
                              void *stream)
{
    clear_error();
    ACO_REQUIRE(n >= 3 && m >= 1 && m <= (1 << 20), "bad sizes n = %d, m = %d", n, m);
    ACO_REQUIRE(tours && lengths && best_len && best_tour, "NULL array argument");
    hipStream_t st = as_stream(stream);
    k_best_copy<<<std::min(1024u, blocks_for(n, 256)), 256, 0, st>>>(tours, lengths, n, m,
                                                                    best_len, best_tour);
    k_best_finish<<<1, 256, 0, st>>>(lengths, m, best_len, iter_best);
    ACO_LAUNCH_CHECK("best tracking");
    return ACO_OK;
}

extern "C" int aco_update_local_best(int32_t n, int32_t m, const int32_t *tours,
                                     const int64_t *lengths, int32_t *lbest, int64_t *lbest_len,
                                     void *stream)
{
    clear_error();
    ACO_REQUIRE(n >= 3 && n <= (1 << 27), "n = %d out of range [3, 2^27]", n);
    ACO_REQUIRE(m >= 1, "m = %d must be >= 1", m);
    ACO_REQUIRE(tours && lengths && lbest && lbest_len, "NULL array argument");
    hipStream_t st = as_stream(stream);
    for (int32_t a0 = 0; a0 < m; a0 += 65535) {
        const int32_t ma = m - a0 < 65535 ? m - a0 : 65535;
        k_lbest_copy<<<dim3(blocks_for(n, 256), (unsigned)ma), 256, 0, st>>>(tours, lengths, n, a0,
                                                                          lbest_len, lbest);
    }
    ACO_LAUNCH_CHECK("k_lbest_copy");
    k_lbest_len<<<blocks_for(m, 256), 256, 0, st>>>(lengths, m, lbest_len);
    ACO_LAUNCH_CHECK("k_lbest_len");
    return ACO_OK;
}

extern "C" int aco_pheromone_local_best(int32_t n, int32_t k, const int32_t *nn,
                                        const int8_t *rev, int32_t m, const int32_t *lbest,
                                        const int64_t *lbest_len, double tau_base, double delta,
                                        int32_t deposit_shift, float *tau, void *ws,
                                        size_t ws_bytes, void *stream)
{
    clear_error();
    ACO_REQUIRE(n >= 3 && n <= (1 << 27), "n = %d out of range [3, 2^27]", n);
    ACO_REQUIRE(k >= 1 && k <= ACO_MAX_K && k <= n - 1, "k = %d out of range", k);
    ACO_REQUIRE(m >= 1, "m = %d must be >= 1", m);
    ACO_REQUIRE(deposit_shift >= 0 && deposit_shift <= 62, "deposit_shift = %d out of [0, 62]",
                deposit_shift);
    // every quantum is at most 2^shift and a slot sums at most m of them
    ACO_REQUIRE((int64_t)m <= (INT64_MAX >> deposit_shift),
                "m * 2^deposit_shift = %d * 2^%d could overflow the int64 sums", m, deposit_shift);
    ACO_REQUIRE(std::isfinite(tau_base) && tau_base >= 0.0 && std::isfinite(delta) && delta >= 0.0,
                "tau_base and delta must be finite and >= 0");
    ACO_REQUIRE(nn && rev && lbest && lbest_len && tau && ws, "NULL array argument");
    const size_t need = aco_update_workspace_bytes(n, k, m);
    if (ws_bytes < need)
        return fail(ACO_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    hipStream_t st = as_stream(stream);
    const int64_t nk = (int64_t)n * k;
    int64_t *acc = (int64_t *)ws;
    int64_t *q = (int64_t *)((char *)ws + (size_t)nk * 8);
    uint32_t *err = device_error_word();
    if (!err) return ACO_ERR_HIP;
    k_zero_i64<<<std::min(4096u, blocks_for(nk, 256)), 256, 0, st>>>(acc, nk);
    k_quanta_ratio<<<1, 1024, 0, st>>>(lbest_len, m, deposit_shift, q, err);
    for (int32_t a0 = 0; a0 < m; a0 += 65535) {
        const int32_t ma = m - a0 < 65535 ? m - a0 : 65535;
        k_deposit<<<dim3(blocks_for(n, 256), (unsigned)ma), 256, 0, st>>>(
            nn, rev, n, k, a0, lbest, nullptr, q, (unsigned long long *)acc, err);
    }
    const float base = (float)tau_base;
    const float scale = (float)(delta * std::ldexp(1.0, -deposit_shift));
    k_merge_base<<<std::min(4096u, blocks_for(nk, 256)), 256, 0, st>>>(tau, acc, nn, rev, k, nk,
                                                                      base, scale);
    ACO_LAUNCH_CHECK("local-best pheromone");
    return ACO_OK;
}
