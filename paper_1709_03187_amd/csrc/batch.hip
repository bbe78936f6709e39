// Batched colonies: thousands of independent TSP instances of uneven size,
// each running the same method (Section 2, Eq. 1-4, on k-NN candidate edges).
//
// Set-up builds, per instance, the grid, the k-NN / 64-NN tables, the
// reverse slots, eta^beta and the nearest-neighbour tour (tau0).  Then ONE
// persistent launch runs all iterations of all instances: one workgroup per
// instance, largest instances first.  Inside a workgroup the waves build the
// instance's ants (ant a on wave a mod W) and then, between workgroup
// barriers, the whole workgroup computes the tour lengths, the iteration
// best, the fixed-point deposit, the merge and the next choice weights.  No
// grid-wide synchronisation is needed, so the launch can be captured in a
// HIP graph and replayed.
//
// The waves per workgroup (W) and the visited-set layout (bits or bytes) are
// tunable; results do not depend on them (ant a always uses Philox counter
// (step, a, iteration) and the update sums integers).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "colony.hpp"
#include "colony_x4.hpp"
#include "common.hpp"

namespace aco {

constexpr int kBatchExt = 64;   // row stride of the batched 64-NN table

struct BatchState {
    const int64_t *off;    // [B+1] city offsets
    const int32_t *order;  // [B] instance of workgroup x (largest first)
    const int32_t *xy;     // [N][2]
    GridHdr *hdr;          // [B]
    int32_t *cell_start;   // instance b at 3 off[b] + 3 b
    int32_t *cursor;       // same layout (build scratch)
    int4 *pts;             // [N], city indices local to the instance
    int32_t *ext;          // [N][64]
    int32_t *nn, *nnd;     // [N][k], local indices
    int8_t *rev;           // [N][k]
    float *eta_b, *tau;    // [N][k]
    CandW *rows;           // [N][row_stride(k)]
    int64_t *acc;          // [N][k]
    int32_t *tours;        // instance b at m off[b]: [m][n_b]
    uint8_t *slots;        // idem
    int64_t *lengths;      // [B][m]
    int32_t *inst_of;      // [N]
    int32_t *flag;         // bit 0: coordinate out of range, bit 1: degenerate instance
    uint32_t *err;         // the device's error word (guards)
    int32_t B, k, m;
};

__device__ __forceinline__ GridView batch_grid(const BatchState &S, int b)
{
    const int64_t off = S.off[b];
    GridView g;
    g.h = S.hdr[b];
    g.cell_start = S.cell_start + 3 * off + 3 * (int64_t)b;
    g.pts = S.pts + off;
    g.ext = S.ext + off * kBatchExt;
    g.ext_stride = kBatchExt;
    g.pinv = nullptr;     // batched colonies work on city indices
    g.ext_pos = nullptr;
    g.ext_pos_stride = 0;
    return g;
}

__global__ void k_set_i32(int32_t *p, int32_t v)
{
    if (threadIdx.x == 0) *p = v;
}

__device__ inline int64_t isqrt_ceil_dev(int64_t v)
{
    if (v <= 0) return 0;
    int64_t r = (int64_t)sqrt((double)v);
    while (r > 0 && (r - 1) * (r - 1) >= v) --r;
    while (r * r < v) ++r;
    return r;
}

// ------------------------------------------------------------------ set-up

// Grid of one instance per workgroup of 256 threads: bounding box, cell side
// (about two cities per cell, at most n cells along a side), counts,
// exclusive scan, scatter (same sizing rule as the single-instance grid).
constexpr int kGridThreads = 256;

__global__ __launch_bounds__(kGridThreads) void k_b_grid(BatchState S)
{
    __shared__ int32_t red[4][kGridThreads / kWave];
    __shared__ GridHdr H;
    __shared__ int32_t part[kGridThreads];
    const int b = blockIdx.x, tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
    const int64_t off = S.off[b];
    const int32_t n = (int32_t)(S.off[b + 1] - off);
    const int32_t *xy = S.xy + 2 * off;
    int32_t mnx = INT32_MAX, mny = INT32_MAX, mxx = INT32_MIN, mxy = INT32_MIN, bad = 0;
    for (int i = tid; i < n; i += kGridThreads) {
        const int32_t x = xy[2 * i], y = xy[2 * i + 1];
        mnx = min(mnx, x);
        mny = min(mny, y);
        mxx = max(mxx, x);
        mxy = max(mxy, y);
        bad |= (x > ACO_COORD_LIMIT || x < -ACO_COORD_LIMIT || y > ACO_COORD_LIMIT ||
                y < -ACO_COORD_LIMIT);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mnx = min(mnx, __shfl_xor(mnx, o));
        mny = min(mny, __shfl_xor(mny, o));
        mxx = max(mxx, __shfl_xor(mxx, o));
        mxy = max(mxy, __shfl_xor(mxy, o));
        bad |= __shfl_xor(bad, o);
    }
    if (lane == 0) {
        red[0][wv] = mnx;
        red[1][wv] = mny;
        red[2][wv] = mxx;
        red[3][wv] = mxy;
        if (bad) atomicOr(S.flag, 1);
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kGridThreads / kWave; ++w) {
            red[0][0] = min(red[0][0], red[0][w]);
            red[1][0] = min(red[1][0], red[1][w]);
            red[2][0] = max(red[2][0], red[2][w]);
            red[3][0] = max(red[3][0], red[3][w]);
        }
        const int64_t W = (int64_t)red[2][0] - red[0][0] + 1, Hh = (int64_t)red[3][0] - red[1][0] + 1;
        if (W == 1 && Hh == 1) atomicOr(S.flag, 2);
        const int64_t target = n / 2 > 0 ? n / 2 : 1;
        int64_t cell = isqrt_ceil_dev((W * Hh + target - 1) / target);
        const int64_t side = W > Hh ? W : Hh;
        cell = max(cell, (side + n - 1) / n);
        cell = max(cell, (int64_t)1);
        H.x0 = red[0][0];
        H.y0 = red[1][0];
        H.cell = (int32_t)cell;
        H.gw = (int32_t)((W + cell - 1) / cell);
        H.gh = (int32_t)((Hh + cell - 1) / cell);
        H.ncell = H.gw * H.gh;
        H.n = n;
        H.cap = 3 * n + 3;
        H.kx = ext_width(n);
        H.kxp = 0;   // no table by position: the batch works on city indices
        S.hdr[b] = H;
    }
    __syncthreads();
    const GridHdr h = H;
    int32_t *cs = S.cell_start + 3 * off + 3 * (int64_t)b;
    int32_t *cur = S.cursor + 3 * off + 3 * (int64_t)b;
    const int32_t len = h.ncell + 1;   // <= n/2 + 2n + 2 < 3n + 3
    for (int c = tid; c < len; c += kGridThreads) cs[c] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += kGridThreads)
        atomicAdd(&cs[cell_y(h, xy[2 * i + 1]) * h.gw + cell_x(h, xy[2 * i])], 1);
    __syncthreads();
    // exclusive scan: each thread owns a contiguous strip
    const int strip = (len + kGridThreads - 1) / kGridThreads;
    const int lo = min(len, tid * strip), hi = min(len, lo + strip);
    int32_t s = 0;
    for (int c = lo; c < hi; ++c) s += cs[c];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < kGridThreads; o <<= 1) {
        const int32_t add = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    int32_t run = part[tid] - s;
    for (int c = lo; c < hi; ++c) {
        const int32_t v = cs[c];
        cs[c] = run;
        cur[c] = run;
        run += v;
    }
    __syncthreads();
    for (int i = tid; i < n; i += kGridThreads) {
        const int32_t x = xy[2 * i], y = xy[2 * i + 1];
        const int pos = atomicAdd(&cur[cell_y(h, y) * h.gw + cell_x(h, x)], 1);
        S.pts[off + pos] = make_int4(x, y, i, 0);
    }
}

// 64-NN and candidate lists of one instance per workgroup of 64 threads
// (threads loop over the instance's cities in grid order).
__global__ __launch_bounds__(kWave) void k_b_knn(BatchState S)
{
    __shared__ uint64_t lists[kBatchExt * kWave];
    const int b = blockIdx.x;
    const int64_t off = S.off[b];
    const int32_t n = (int32_t)(S.off[b + 1] - off);
    const GridView g = batch_grid(S, b);
    const int kx = g.h.kx, k = S.k;
    uint64_t *L = lists + threadIdx.x;
    for (int p = threadIdx.x; p < n; p += kWave) {
        const int4 me = g.pts[p];
        knn_city(g, me, kx, L, kWave);
        const int64_t row = (off + me.z) * k, xrow = (off + me.z) * kBatchExt;
        for (int r = 0; r < kx; ++r) {
            const uint64_t key = L[(int64_t)r * kWave];
            S.ext[xrow + r] = (int32_t)(uint32_t)key;
            if (r < k) {
                S.nn[row + r] = (int32_t)(uint32_t)key;
                S.nnd[row + r] = (int32_t)(key >> 32);
            }
        }
        S.inst_of[off + me.z] = b;
    }
}

// rev and eta^beta of every candidate slot (thread per slot).
__global__ void k_b_rev_eta(BatchState S, int64_t slots_total, double beta)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= slots_total) return;
    const int k = S.k;
    const int64_t gi = e / k;
    const int b = S.inst_of[gi];
    const int64_t off = S.off[b];
    const int32_t i = (int32_t)(gi - off);
    const int64_t rj = (off + S.nn[e]) * k;
    int8_t out = -1;
    for (int s = 0; s < k; ++s)
        if (S.nn[rj + s] == i) {
            out = (int8_t)s;
            break;
        }
    S.rev[e] = out;
    const int32_t d = S.nnd[e];
    const double eta = 1.0 / (double)(d > 1 ? d : 1);
    S.eta_b[e] = (float)(beta == 0.0 ? 1.0 : (beta == 1.0 ? eta : pow(eta, beta)));
}

// Nearest-neighbour tour, tau0 = fl32(1/(n L_nn)) and the first choice
// weights of one instance per wave; the best so far starts as the NN tour.
__global__ __launch_bounds__(kWave) void k_b_init(BatchState S, double alpha,
                                                  int32_t *best_tours, int64_t *best_lens)
{
    extern __shared__ uint32_t vis[];
    const int b = blockIdx.x, lane = lane_id(), k = S.k;
    const int64_t off = S.off[b];
    const int32_t n = (int32_t)(S.off[b + 1] - off);
    const int64_t L = nn_tour_wave(S.xy + 2 * off, n, k, S.nn + off * k, S.nnd + off * k,
                                   batch_grid(S, b), VisBits{vis}, best_tours + off, S.err);
    if (L <= 0) {
        if (lane == 0) atomicOr(S.flag, 2);
        return;
    }
    if (lane == 0) best_lens[b] = L;
    const float t0 = (float)(1.0 / ((double)n * (double)L));
    for (int64_t e = lane; e < (int64_t)n * k; e += kWave) S.tau[off * k + e] = t0;
    __syncthreads();   // the rows below read tau written by other lanes
    for (int i = lane; i < n; i += kWave) {
        const int64_t rb = (off + i) * k;
        choice_row(S.nn + rb, S.tau + rb, S.eta_b + rb, k, alpha,
                   S.rows + (off + i) * row_stride(k));
    }
}

// ------------------------------------------------------------------ the persistent colony

struct ColonyParams {
    double alpha;
    float evap;      // fl32(1 - rho)
    float scale;     // 2^-shift
    int32_t shift;
    uint64_t seed;
    int32_t first_iteration, count;
    size_t vis_stride;   // LDS bytes per wave for the visited set(s)
    size_t set_bytes;    // four ants per wave: bytes of one ant's visited bitmask
    int32_t *best_tours; // [N]
    int64_t *best_lens;  // [B]
    int64_t *iter_best;  // row b at iter_best + b * ib_stride, or nullptr
    int32_t ib_stride;
    float *step_prob;    // [N * m] as tours (one ant per wave only), or nullptr
};

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int64_t wave_min_i64_shfl(int64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t u = __shfl_xor(v, o);
        v = u < v ? u : v;
    }
    return v;
}

// OCC = waves per SIMD the register allocation must allow (4: up to 128
// VGPRs; 8: 64 VGPRs, spilling on the rare fallback path): the ants resident
// per CU, one of the tuned knobs.  APW = ants per wave: 1 (build_ant) or 4
// (build_ants4, k <= 16, bit visited sets); the tours are the same.
template <int KP, class Vis, int OCC, int APW>
__global__ __launch_bounds__(1024, OCC) void k_b_colony(BatchState S, ColonyParams P)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int32_t win;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int W = blockDim.x / kWave, nthr = blockDim.x;
    const int b = S.order[blockIdx.x];
    const int k = S.k, m = S.m;
    const int64_t off = S.off[b];
    const int32_t n = (int32_t)(S.off[b + 1] - off);
    const int32_t *xy = S.xy + 2 * off;
    const int32_t *nn = S.nn + off * k;
    const int8_t *rev = S.rev + off * k;
    const float *eta_b = S.eta_b + off * k;
    float *tau = S.tau + off * k;
    CandW *rows = S.rows + off * row_stride(k);
    int64_t *acc = S.acc + off * k;
    int32_t *tours = S.tours + off * m;
    uint8_t *slots = S.slots + off * m;
    int64_t *lens = S.lengths + (int64_t)b * m;
    int64_t *q = (int64_t *)(lds + (size_t)W * P.vis_stride);   // [m]
    const Vis vis = Vis::at(lds + (size_t)wave * P.vis_stride);
    const int32_t nk = n * k;

    for (int it = 0; it < P.count; ++it) {
        const uint32_t t = (uint32_t)(P.first_iteration + it);
        // 1. construction: ant a on wave a mod W (four at a time: a, a + W,
        //    a + 2W, a + 3W on one wave)
        if constexpr (APW == 4) {
            unsigned char *mine = lds + (size_t)wave * P.vis_stride;
            for (int a0 = wave; a0 < m; a0 += 4 * W) {
                Ants4Task T4;
                T4.xy = xy;
                T4.rows = rows;
                T4.n = n;
                T4.k = k;
                T4.ant0 = (uint32_t)a0;
                T4.ant_stride = (uint32_t)W;
                int nv = 1;
                while (nv < 4 && a0 + nv * W < m) ++nv;
                T4.nvalid = nv;
                T4.iteration = t;
                T4.seed = P.seed;
                T4.tours = tours;
                T4.slots = slots;
                T4.err = S.err;
                build_ants4(T4, mine, P.set_bytes, [&]() { return batch_grid(S, b); });
            }
        } else
        for (int a = wave; a < m; a += W) {
            AntTask T;
            T.xy = xy;
            T.rows = rows;
            T.n = n;
            T.k = k;
            T.ant = (uint32_t)a;
            T.iteration = t;
            T.seed = P.seed;
            T.tour = tours + (int64_t)a * n;
            T.slots = slots + (int64_t)a * n;
            T.prob = P.step_prob ? P.step_prob + off * m + (int64_t)a * n : nullptr;
            T.err = S.err;
            build_ant<KP>(T, vis, [&]() { return batch_grid(S, b); });
        }
        __syncthreads();
        // 2. exact tour lengths, one wave per ant
        for (int a = wave; a < m; a += W) {
            const int32_t *T = tours + (int64_t)a * n;
            int64_t d = 0;
            for (int e = lane; e < n; e += kWave) {
                const int32_t i = T[e], j = T[e + 1 == n ? 0 : e + 1];
                d += nint_sqrt(sq_dist(xy[2 * i], xy[2 * i + 1], xy[2 * j], xy[2 * j + 1]));
            }
            d = wave_sum_i64(d);
            if (lane == 0) lens[a] = d;
        }
        __syncthreads();
        // 3. iteration best (lowest ant on ties) and the per-ant deposit quanta
        if (wave == 0) {
            int64_t lmin = INT64_MAX;
            for (int a = lane; a < m; a += kWave) lmin = lens[a] < lmin ? lens[a] : lmin;
            lmin = wave_min_i64_shfl(lmin);
            int64_t amin = INT64_MAX;
            for (int a = lane; a < m; a += kWave)
                if (lens[a] == lmin && a < amin) amin = a;
            amin = wave_min_i64_shfl(amin);
            if (lane == 0) {
                if (P.iter_best) P.iter_best[(int64_t)b * P.ib_stride + it] = lmin;
                const bool better = lmin < P.best_lens[b];
                if (better) P.best_lens[b] = lmin;
                win = better ? (int32_t)amin : -1;
            }
        }
        for (int a = tid; a < m; a += nthr) {
            const int64_t L = lens[a];
            q[a] = L > 0 ? ((int64_t)1 << P.shift) / L : 0;
        }
        for (int e = tid; e < nk; e += nthr) acc[e] = 0;
        __syncthreads();
        if (win >= 0)
            for (int e = tid; e < n; e += nthr)
                P.best_tours[off + e] = tours[(int64_t)win * n + e];
        // 4. deposit: one int64 atomic per undirected candidate edge (canonical slot)
        for (int64_t e = tid; e < (int64_t)m * n; e += nthr) {
            const int32_t a = (int32_t)((uint32_t)e / (uint32_t)n);
            const int32_t s = (int32_t)(e - (int64_t)a * n);
            const int32_t *T = tours + (int64_t)a * n;
            const int32_t i = T[s], j = T[s + 1 == n ? 0 : s + 1];
            const int64_t ri = (int64_t)i * k, rj = (int64_t)j * k;
            int r = -1;
            if (s + 1 < n) {
                const uint32_t sl = slots[(int64_t)a * n + s + 1];
                if (sl < (uint32_t)k) r = (int)sl;
            }
            if (r < 0)
                for (int x = 0; x < k; ++x)
                    if (nn[ri + x] == j) { r = x; break; }
            int r2 = -1;
            if (r >= 0) r2 = rev[ri + r];
            else
                for (int x = 0; x < k; ++x)
                    if (nn[rj + x] == i) { r2 = x; break; }
            // one atomic on the selected slot (two guarded atomics compile to
            // two masked atomic instructions per edge)
            const int64_t dst = (r >= 0 && (r2 < 0 || i < j)) ? ri + r
                              : (r2 >= 0 && r2 < k)           ? rj + r2
                                                              : -1;
            if (dst >= 0) atomicAdd((unsigned long long *)&acc[dst], (unsigned long long)q[a]);
        }
        __syncthreads();
        // 5. merge (evaporation, then the deposit of the slot's canonical
        //    slot) fused with the next iteration's choice weights: one lane per
        //    slot, an aligned group of KP lanes per row, so each row's weights
        //    are formed from the merged values in registers.  acc was updated by
        //    L2 atomics: read it with device-coherent loads.  Every lane of a
        //    wave runs the same trips (the row maximum uses cross-lane moves).
        for (int64_t base = (int64_t)wave * kWave; base < (int64_t)n * KP; base += nthr) {
            const int64_t t = base + lane;
            const int32_t i = (int32_t)(t / KP);
            const int r = (int)(t % KP);
            const bool act = i < n && r < k;
            float tv = 0.0f, eb = 0.0f;
            int32_t j = 0;
            if (act) {
                const int64_t e = (int64_t)i * k + r;
                j = nn[e];
                const int r2 = rev[e];
                const int64_t src = (r2 >= 0 && j < i) ? (int64_t)j * k + r2 : e;
                const int64_t a64 = __hip_atomic_load(&acc[src], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                const float ev = __fmul_rn(tau[e], P.evap);
                const float dep = __fmul_rn((float)a64, P.scale);
                tv = __fadd_rn(ev, dep);
                tau[e] = tv;
                eb = eta_b[e];
            }
            const float w = choice_weight_lane<KP>(act, tv, eb, P.alpha);
            if (act) rows[(int64_t)i * row_stride(KP) + r] = CandW{j, w};
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host side

struct BatchLayoutHost {
    size_t off, order, hdr, cell_start, cursor, pts, ext, nn, nnd, rev, eta_b, tau, rows, acc,
        tours, slots, lengths, inst_of, flag, total;
    int64_t N, nmax;
};

static bool batch_layout(const int64_t *offs, int32_t B, int32_t k, int32_t m, BatchLayoutHost &L)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t N = offs[B];
    int64_t nmax = 0;
    for (int b = 0; b < B; ++b) nmax = std::max(nmax, offs[b + 1] - offs[b]);
    L.N = N;
    L.nmax = nmax;
    size_t o = 0;
    L.off = o;        o = al(o + (size_t)(B + 1) * 8);
    L.order = o;      o = al(o + (size_t)B * 4);
    L.hdr = o;        o = al(o + (size_t)B * sizeof(GridHdr));
    L.cell_start = o; o = al(o + (size_t)(3 * N + 3 * (int64_t)B) * 4);
    L.cursor = o;     o = al(o + (size_t)(3 * N + 3 * (int64_t)B) * 4);
    L.pts = o;        o = al(o + (size_t)N * 16);
    L.ext = o;        o = al(o + (size_t)N * kBatchExt * 4);
    L.nn = o;         o = al(o + (size_t)N * k * 4);
    L.nnd = o;        o = al(o + (size_t)N * k * 4);
    L.rev = o;        o = al(o + (size_t)N * k);
    L.eta_b = o;      o = al(o + (size_t)N * k * 4);
    L.tau = o;        o = al(o + (size_t)N * k * 4);
    L.rows = o;       o = al(o + (size_t)N * row_stride(k) * sizeof(CandW));
    L.acc = o;        o = al(o + (size_t)N * k * 8);
    L.tours = o;      o = al(o + (size_t)N * m * 4);
    L.slots = o;      o = al(o + (size_t)N * m);
    L.lengths = o;    o = al(o + (size_t)B * m * 8);
    L.inst_of = o;    o = al(o + (size_t)N * 4);
    L.flag = o;       o = al(o + 8);
    L.total = o;
    return true;
}

static BatchState batch_state(void *ws, const BatchLayoutHost &L, const int32_t *xy, int32_t B,
                              int32_t k, int32_t m)
{
    char *w = (char *)ws;
    BatchState S;
    S.off = (const int64_t *)(w + L.off);
    S.order = (const int32_t *)(w + L.order);
    S.xy = xy;
    S.hdr = (GridHdr *)(w + L.hdr);
    S.cell_start = (int32_t *)(w + L.cell_start);
    S.cursor = (int32_t *)(w + L.cursor);
    S.pts = (int4 *)(w + L.pts);
    S.ext = (int32_t *)(w + L.ext);
    S.nn = (int32_t *)(w + L.nn);
    S.nnd = (int32_t *)(w + L.nnd);
    S.rev = (int8_t *)(w + L.rev);
    S.eta_b = (float *)(w + L.eta_b);
    S.tau = (float *)(w + L.tau);
    S.rows = (CandW *)(w + L.rows);
    S.acc = (int64_t *)(w + L.acc);
    S.tours = (int32_t *)(w + L.tours);
    S.slots = (uint8_t *)(w + L.slots);
    S.lengths = (int64_t *)(w + L.lengths);
    S.inst_of = (int32_t *)(w + L.inst_of);
    S.flag = (int32_t *)(w + L.flag);
    S.err = device_error_word();
    S.B = B;
    S.k = k;
    S.m = m;
    return S;
}

static int validate_batch(const int64_t *offs, int32_t B, const aco_params_t *p)
{
    ACO_REQUIRE(p != nullptr && offs != nullptr, "NULL params or offsets");
    if (p->eta_mode != ACO_ETA_DISTANCE)
        return fail(ACO_ERR_UNSUPPORTED, "the batched colonies use eta = 1/d only");
    ACO_REQUIRE(B >= 1 && B <= (1 << 24), "B = %d out of range", B);
    ACO_REQUIRE(offs[0] == 0, "offsets[0] must be 0");
    int64_t nmin = INT64_MAX, nmax = 0;
    for (int b = 0; b < B; ++b) {
        const int64_t nb = offs[b + 1] - offs[b];
        nmin = std::min(nmin, nb);
        nmax = std::max(nmax, nb);
    }
    ACO_REQUIRE(nmin >= 3, "every instance needs n >= 3 (smallest has %lld)", (long long)nmin);
    ACO_REQUIRE(nmax <= 65536, "batched instances are limited to n <= 65536 (largest %lld)",
                (long long)nmax);
    ACO_REQUIRE(offs[B] <= (int64_t)INT32_MAX / 64, "too many cities in the batch");
    ACO_REQUIRE(p->k >= 1 && p->k <= ACO_MAX_K && p->k <= nmin - 1,
                "k = %d must be in [1, min(64, smallest n - 1)]", p->k);
    ACO_REQUIRE(p->m >= 1 && p->m <= 1024, "m = %d out of range [1, 1024]", p->m);
    ACO_REQUIRE(std::isfinite(p->alpha) && p->alpha >= 0, "alpha must be finite and >= 0");
    ACO_REQUIRE(std::isfinite(p->beta) && p->beta >= 0, "beta must be finite and >= 0");
    ACO_REQUIRE(p->rho > 0.0 && p->rho <= 1.0, "rho must lie in (0, 1]");
    ACO_REQUIRE(p->iterations >= 0, "iterations must be >= 0");
    ACO_REQUIRE(p->deposit_shift >= 0 && p->deposit_shift <= 62, "deposit_shift out of [0, 62]");
    return ACO_OK;
}

using ColonyKernel = void (*)(BatchState, ColonyParams);

template <class Vis, int OCC>
static ColonyKernel colony_kernel_k(int k)
{
    return k <= 8 ? k_b_colony<8, Vis, OCC, 1> : k <= 16 ? k_b_colony<16, Vis, OCC, 1>
           : k <= 32 ? k_b_colony<32, Vis, OCC, 1> : k_b_colony<64, Vis, OCC, 1>;
}

static ColonyKernel colony_kernel(int k, int layout, int occ)
{
    if (layout == ACO_VIS_BITS_X4)   // k <= 16 (checked by the callers)
        return occ == 8 ? (k <= 8 ? k_b_colony<8, VisBits, 8, 4> : k_b_colony<16, VisBits, 8, 4>)
                        : (k <= 8 ? k_b_colony<8, VisBits, 4, 4> : k_b_colony<16, VisBits, 4, 4>);
    if (layout == ACO_VIS_BYTES)
        return occ == 8 ? colony_kernel_k<VisBytes, 8>(k) : colony_kernel_k<VisBytes, 4>(k);
    return occ == 8 ? colony_kernel_k<VisBits, 8>(k) : colony_kernel_k<VisBits, 4>(k);
}

// Bytes of one ant's bit visited set, padded to 16.
static size_t set_bytes_bits(int64_t nmax)
{
    return ((size_t)((nmax + 31) / 32) * 4 + 15) & ~(size_t)15;
}

static size_t vis_stride(int layout, int64_t nmax)
{
    if (layout == ACO_VIS_BITS_X4)
        return (ants4_lds_bytes(set_bytes_bits(nmax)) + 15) & ~(size_t)15;
    const size_t b = layout == ACO_VIS_BYTES ? (size_t)((nmax + 3) & ~3) : (size_t)((nmax + 31) / 32) * 4;
    return (b + 15) & ~(size_t)15;
}

static size_t colony_lds(int waves, int layout, int64_t nmax, int m)
{
    return (size_t)waves * vis_stride(layout, nmax) + (size_t)m * 8;
}

// A launch configuration: waves per instance workgroup, visited-set layout,
// waves per SIMD the registers allow.  None of them changes the results.
struct Tuning {
    int waves, layout, occ;
};

// The shape used before (or without) tuning: four ants per wave with as many
// waves per instance as the LDS holds when k <= 16, else one ant per wave.
static Tuning default_tuning(int k, int64_t nmax, int m)
{
    if (k <= 16)
        for (int w : {16, 8, 4})
            if (colony_lds(w, ACO_VIS_BITS_X4, nmax, m) <= max_lds_per_block())
                return Tuning{w, ACO_VIS_BITS_X4, 8};
    return Tuning{8, ACO_VIS_BITS, 4};
}

// Tuned configuration per (device, k, m, largest n, batch size).
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int64_t, int>, Tuning> g_tuned;

static int launch_colony(const BatchState &S0, const BatchLayoutHost &L, const aco_params_t *p,
                         int32_t first, int32_t count, Tuning cfg, int32_t *best_tours,
                         int64_t *best_lens, int64_t *iter_best, int32_t ib_stride, hipStream_t st,
                         float *step_prob = nullptr)
{
    if (S0.xy == nullptr || best_tours == nullptr || best_lens == nullptr)
        return fail(ACO_ERR_INVALID_ARG, "NULL coordinates or outputs for the colony launch");
    const int waves = cfg.waves, layout = cfg.layout;
    const size_t lds = colony_lds(waves, layout, L.nmax, p->m);
    if (lds > max_lds_per_block())
        return fail(ACO_ERR_UNSUPPORTED, "batched LDS of %zu bytes exceeds the limit", lds);
    ColonyKernel kern = colony_kernel(p->k, layout, cfg.occ);
    if (lds > 65536)
        ACO_HIP_CHECK(hipFuncSetAttribute((const void *)kern,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ColonyParams P;
    P.alpha = p->alpha;
    P.evap = (float)(1.0 - p->rho);
    P.scale = std::ldexp(1.0f, -p->deposit_shift);
    P.shift = p->deposit_shift;
    P.seed = p->seed;
    P.first_iteration = first;
    P.count = count;
    P.vis_stride = vis_stride(layout, L.nmax);
    P.set_bytes = set_bytes_bits(L.nmax);
    P.best_tours = best_tours;
    P.best_lens = best_lens;
    P.iter_best = iter_best;
    P.ib_stride = ib_stride;
    P.step_prob = step_prob;
    kern<<<S0.B, waves * kWave, lds, st>>>(S0, P);
    ACO_LAUNCH_CHECK("k_b_colony");
    return ACO_OK;
}

}  // namespace aco

using namespace aco;

// Candidate counts the k-auto mode compares (those <= min n_b - 1).
static const int kAutoK[] = {8, 10, 12, 16};
static constexpr int kAutoKMax = 16;
static constexpr int kAutoProbe = 8;   // iterations each candidate runs

extern "C" size_t aco_batch_workspace_bytes(const int64_t *offsets, int32_t B,
                                            const aco_params_t *pin)
{
    aco_params_t q;
    if (load_params(pin, q) != ACO_OK) return 0;
    const aco_params_t *p = &q;
    if (!offsets || B < 1 || p->k < 0 || p->m < 1) return 0;
    int k = p->k;
    if (k == 0) {   // k-auto: room for the largest candidate
        int64_t nmin = INT64_MAX;
        for (int b = 0; b < B; ++b) nmin = std::min(nmin, offsets[b + 1] - offsets[b]);
        k = (int)std::max<int64_t>(1, std::min<int64_t>(kAutoKMax, nmin - 1));
    }
    BatchLayoutHost L;
    batch_layout(offsets, B, k, p->m, L);
    return L.total;
}

extern "C" int aco_batch_layout(const int64_t *offsets, int32_t B, const aco_params_t *pin,
                                aco_batch_layout_t *out)
{
    clear_error();
    aco_params_t q;
    int rc = load_params(pin, q);
    if (rc != ACO_OK) return rc;
    const aco_params_t *p = &q;
    rc = validate_batch(offsets, B, p);
    if (rc != ACO_OK) return rc;
    ACO_REQUIRE(out != nullptr, "NULL output");
    BatchLayoutHost L;
    batch_layout(offsets, B, p->k, p->m, L);
    out->nn = L.nn;
    out->nnd = L.nnd;
    out->rev = L.rev;
    out->eta_b = L.eta_b;
    out->tau = L.tau;
    out->tours = L.tours;
    out->slots = L.slots;
    out->lengths = L.lengths;
    out->total = L.total;
    return ACO_OK;
}

extern "C" int aco_batch_setup(const int32_t *xy, const int64_t *offsets, int32_t B,
                               const aco_params_t *pin, int32_t *best_tours, int64_t *best_lens,
                               void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    aco_params_t q;
    int rc = load_params(pin, q);
    if (rc != ACO_OK) return rc;
    const aco_params_t *p = &q;
    rc = validate_batch(offsets, B, p);
    if (rc != ACO_OK) return rc;
    ACO_REQUIRE(xy && best_tours && best_lens && ws, "NULL array argument");
    BatchLayoutHost L;
    batch_layout(offsets, B, p->k, p->m, L);
    if (ws_bytes < L.total)
        return fail(ACO_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    const size_t lds_init = bitmask_bytes(L.nmax);
    if (lds_init > max_lds_per_block())
        return fail(ACO_ERR_UNSUPPORTED, "visited bitmask exceeds LDS");
    hipStream_t st = as_stream(stream);
    BatchState S = batch_state(ws, L, xy, B, p->k, p->m);
    // offsets and the largest-first processing order
    std::vector<int32_t> order(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
    });
    char *w = (char *)ws;
    ACO_HIP_CHECK(hipMemcpyAsync(w + L.off, offsets, (size_t)(B + 1) * 8, hipMemcpyHostToDevice, st));
    ACO_HIP_CHECK(hipMemcpyAsync(w + L.order, order.data(), (size_t)B * 4, hipMemcpyHostToDevice, st));
    k_set_i32<<<1, 64, 0, st>>>(S.flag, 0);
    k_b_grid<<<B, kGridThreads, 0, st>>>(S);
    k_b_knn<<<B, kWave, 0, st>>>(S);
    const int64_t slots_total = L.N * p->k;
    k_b_rev_eta<<<blocks_for(slots_total, 256), 256, 0, st>>>(S, slots_total, p->beta);
    k_b_init<<<B, kWave, lds_init, st>>>(S, p->alpha, best_tours, best_lens);
    ACO_LAUNCH_CHECK("batched set-up");
    int32_t flag = 0;
    ACO_HIP_CHECK(hipMemcpyAsync(&flag, S.flag, 4, hipMemcpyDeviceToHost, st));
    ACO_HIP_CHECK(hipStreamSynchronize(st));
    rc = report_device_error(st);
    if (rc != ACO_OK) return rc;
    if (flag & 1) return fail(ACO_ERR_INVALID_ARG, "a coordinate exceeds +-%d", ACO_COORD_LIMIT);
    if (flag & 2) return fail(ACO_ERR_DEGENERATE, "an instance has all its cities coincident");
    return ACO_OK;
}

extern "C" int aco_batch_iterate(const int32_t *xy, const int64_t *offsets, int32_t B,
                                 const aco_params_t *pin, int32_t first_iteration, int32_t count,
                                 int32_t waves, int32_t vis_layout, int32_t occupancy,
                                 int32_t *best_tours, int64_t *best_lens, int64_t *iter_best,
                                 float *step_prob, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    aco_params_t q;
    int rc = load_params(pin, q);
    if (rc != ACO_OK) return rc;
    const aco_params_t *p = &q;
    rc = validate_batch(offsets, B, p);
    if (rc != ACO_OK) return rc;
    ACO_REQUIRE(xy && best_tours && best_lens && ws, "NULL array argument");
    ACO_REQUIRE(first_iteration >= 0 && count >= 0, "bad iteration range");
    ACO_REQUIRE(waves == 0 || waves == 1 || waves == 2 || waves == 4 || waves == 8 || waves == 16,
                "waves per instance must be 0 (tuned), 1, 2, 4, 8 or 16");
    ACO_REQUIRE(vis_layout == 0 || vis_layout == ACO_VIS_BITS || vis_layout == ACO_VIS_BYTES ||
                    vis_layout == ACO_VIS_BITS_X4,
                "bad visited-set layout");
    ACO_REQUIRE(vis_layout != ACO_VIS_BITS_X4 || p->k <= 16,
                "four ants per wave need k <= 16 (k = %d)", p->k);
    ACO_REQUIRE(occupancy == 0 || occupancy == 4 || occupancy == 8,
                "occupancy must be 0 (tuned), 4 or 8 waves per SIMD");
    ACO_REQUIRE(!step_prob || vis_layout != ACO_VIS_BITS_X4,
                "step probabilities are recorded with one ant per wave only");
    BatchLayoutHost L;
    batch_layout(offsets, B, p->k, p->m, L);
    if (ws_bytes < L.total)
        return fail(ACO_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (count == 0) return ACO_OK;
    int dev = 0;
    (void)hipGetDevice(&dev);
    Tuning cfg = default_tuning(p->k, L.nmax, p->m);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(std::make_tuple(dev, p->k, p->m, L.nmax, B));
        if (it != g_tuned.end()) cfg = it->second;
    }
    if (waves) cfg.waves = waves;
    if (vis_layout) cfg.layout = vis_layout;
    if (occupancy) cfg.occ = occupancy;
    // a given wave count with the default four-ant layout may not fit in LDS:
    // then one ant per wave
    if (!vis_layout && cfg.layout == ACO_VIS_BITS_X4 &&
        (step_prob || colony_lds(cfg.waves, cfg.layout, L.nmax, p->m) > max_lds_per_block()))
        cfg.layout = ACO_VIS_BITS;
    BatchState S = batch_state(ws, L, xy, B, p->k, p->m);
    return launch_colony(S, L, p, first_iteration, count, cfg, best_tours, best_lens, iter_best,
                         count, as_stream(stream), step_prob);
}

// Device state that a batched iteration reads and changes: the pheromone, the
// choice weights, the best tours and their lengths.  Held in stream-ordered
// memory so that every tuning candidate starts from the same state.
struct BatchSnapshot {
    char *mem = nullptr;
    size_t tau = 0, rows = 0, bt = 0, bl = 0, total = 0;
};

static int snapshot_alloc(BatchSnapshot &s, const BatchLayoutHost &L, int k, int B,
                          hipStream_t st)
{
    s.tau = (size_t)L.N * k * 4;
    s.rows = (size_t)L.N * row_stride(k) * sizeof(CandW);
    s.bt = (size_t)L.N * 4;
    s.bl = (size_t)B * 8;
    s.total = s.tau + s.rows + s.bt + s.bl;
    ACO_HIP_CHECK(hipMallocAsync((void **)&s.mem, s.total, st));
    return ACO_OK;
}

static int snapshot_copy(const BatchSnapshot &s, const BatchState &S, int32_t *best_tours,
                         int64_t *best_lens, bool take, hipStream_t st)
{
    char *m = s.mem;
    void *dev[4] = {S.tau, S.rows, best_tours, best_lens};
    const size_t len[4] = {s.tau, s.rows, s.bt, s.bl};
    for (int i = 0; i < 4; ++i) {
        if (take)
            ACO_HIP_CHECK(hipMemcpyAsync(m, dev[i], len[i], hipMemcpyDeviceToDevice, st));
        else
            ACO_HIP_CHECK(hipMemcpyAsync(dev[i], m, len[i], hipMemcpyDeviceToDevice, st));
        m += len[i];
    }
    return ACO_OK;
}

// Shape tuning: every candidate runs iteration 0 from the state left by the
// set-up (restored before each), timed with events; the state is restored
// once more at the end.  The fastest shape is cached per device and shape.
static int tune_shape(const BatchState &S, const BatchLayoutHost &L, const aco_params_t *p,
                      int32_t *best_tours, int64_t *best_lens, hipStream_t st, Tuning &best)
{
    const Tuning cand[] = {{4, ACO_VIS_BITS, 4},     {8, ACO_VIS_BITS, 4},
                           {16, ACO_VIS_BITS, 4},    {4, ACO_VIS_BYTES, 4},
                           {8, ACO_VIS_BYTES, 4},    {16, ACO_VIS_BYTES, 4},
                           {4, ACO_VIS_BITS, 8},     {8, ACO_VIS_BITS, 8},
                           {16, ACO_VIS_BITS, 8},    {8, ACO_VIS_BYTES, 8},
                           {4, ACO_VIS_BITS_X4, 4},  {8, ACO_VIS_BITS_X4, 4},
                           {16, ACO_VIS_BITS_X4, 4}, {4, ACO_VIS_BITS_X4, 8},
                           {8, ACO_VIS_BITS_X4, 8},  {16, ACO_VIS_BITS_X4, 8}};
    BatchSnapshot snap;
    int rc = snapshot_alloc(snap, L, p->k, S.B, st);
    if (rc != ACO_OK) return rc;
    rc = snapshot_copy(snap, S, best_tours, best_lens, true, st);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == ACO_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(ACO_ERR_HIP, "hipEventCreate failed");
    float best_ms = 1e30f;
    for (const Tuning &c : cand) {
        if (rc != ACO_OK) break;
        if (colony_lds(c.waves, c.layout, L.nmax, p->m) > max_lds_per_block()) continue;
        if (c.layout == ACO_VIS_BITS_X4 && p->k > 16) continue;
        rc = snapshot_copy(snap, S, best_tours, best_lens, false, st);
        if (rc != ACO_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(ACO_ERR_HIP, "event"); break; }
        rc = launch_colony(S, L, p, 0, 1, c, best_tours, best_lens, nullptr, 1, st);
        if (rc != ACO_OK) break;
        float ms = 0;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(ACO_ERR_HIP, "timing a tuning candidate failed");
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    if (rc == ACO_OK) rc = snapshot_copy(snap, S, best_tours, best_lens, false, st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    const hipError_t fe = hipFreeAsync(snap.mem, st);
    if (rc == ACO_OK && fe != hipSuccess) rc = fail(ACO_ERR_HIP, "hipFreeAsync failed");
    return rc;
}

// k-auto: every candidate k runs the set-up and min(iterations, 8)
// iterations; its quality after i iterations is the mean over instances of
// (best so far, the NN tour included) / (NN-tour length), which does not
// depend on k.  The target is the worst final quality among the candidates,
// which every candidate reaches; the chosen k reaches it in the least time
// (iterations needed times its measured time per iteration; ties to the
// smaller k).
static int choose_k(const int32_t *xy, const int64_t *offsets, int32_t B, const aco_params_t *p,
                    int32_t *best_tours, int64_t *best_lens, void *ws, size_t ws_bytes,
                    void *stream, int &k_out)
{
    hipStream_t st = as_stream(stream);
    int64_t nmin = INT64_MAX;
    for (int b = 0; b < B; ++b) nmin = std::min(nmin, offsets[b + 1] - offsets[b]);
    const int P = std::max(1, std::min(p->iterations, kAutoProbe));
    std::vector<int> ks;
    for (int k : kAutoK)
        if (k <= nmin - 1) ks.push_back(k);
    if (ks.empty()) ks.push_back((int)std::max<int64_t>(1, std::min<int64_t>(nmin - 1, kAutoKMax)));
    std::vector<std::vector<double>> quality(ks.size(), std::vector<double>(P));
    std::vector<double> per_iter_ms(ks.size());
    int64_t *ib = nullptr;
    ACO_HIP_CHECK(hipMallocAsync((void **)&ib, (size_t)B * P * 8, st));
    std::vector<int64_t> L0(B), hib((size_t)B * P);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ACO_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = fail(ACO_ERR_HIP, "hipEventCreate failed");
    for (size_t c = 0; c < ks.size() && rc == ACO_OK; ++c) {
        aco_params_t q = *p;
        q.k = ks[c];
        q.iterations = P;
        rc = aco_batch_setup(xy, offsets, B, &q, best_tours, best_lens, ws, ws_bytes, stream);
        if (rc != ACO_OK) break;
        if (hipMemcpyAsync(L0.data(), best_lens, (size_t)B * 8, hipMemcpyDeviceToHost, st) !=
            hipSuccess) { rc = fail(ACO_ERR_HIP, "copy"); break; }
        BatchLayoutHost L;
        batch_layout(offsets, B, q.k, q.m, L);
        const BatchState S = batch_state(ws, L, xy, B, q.k, q.m);
        if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(ACO_ERR_HIP, "event"); break; }
        rc = launch_colony(S, L, &q, 0, P, default_tuning(q.k, L.nmax, q.m), best_tours,
                           best_lens, ib, P, st);
        if (rc != ACO_OK) break;
        float ms = 0;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
            hipMemcpy(hib.data(), ib, (size_t)B * P * 8, hipMemcpyDeviceToHost) != hipSuccess) {
            rc = fail(ACO_ERR_HIP, "timing a k candidate failed");
            break;
        }
        per_iter_ms[c] = ms / P;
        std::vector<int64_t> sofar(L0);
        for (int i = 0; i < P; ++i) {
            double acc = 0.0;
            for (int b = 0; b < B; ++b) {
                sofar[b] = std::min(sofar[b], hib[(size_t)b * P + i]);
                acc += (double)sofar[b] / (double)L0[b];
            }
            quality[c][i] = acc / B;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    const hipError_t fe = hipFreeAsync(ib, st);
    if (rc != ACO_OK) return rc;
    if (fe != hipSuccess) return fail(ACO_ERR_HIP, "hipFreeAsync failed");
    double target = 0.0;
    for (size_t c = 0; c < ks.size(); ++c) target = std::max(target, quality[c][P - 1]);
    double best_t = 1e300;
    k_out = ks[0];
    for (size_t c = 0; c < ks.size(); ++c) {
        int i = 0;
        while (i < P - 1 && quality[c][i] > target) ++i;
        const double t = (i + 1) * per_iter_ms[c];
        if (t < best_t) {
            best_t = t;
            k_out = ks[c];
        }
    }
    return ACO_OK;
}

extern "C" int aco_run_batched(const int32_t *xy, const int64_t *offsets, int32_t B,
                               const aco_params_t *p, int32_t autotune, int32_t *best_tours,
                               int64_t *best_lens, int64_t *iter_best, void *ws, size_t ws_bytes,
                               void *stream, int32_t *tuned_out)
{
    clear_error();
    aco_params_t q;
    int rc = load_params(p, q);
    if (rc != ACO_OK) return rc;
    if (q.k == 0) {   // k-auto: the workspace is sized for the largest candidate
        aco_params_t big = q;
        big.k = 1;
        rc = validate_batch(offsets, B, &big);
        if (rc != ACO_OK) return rc;
        ACO_REQUIRE(xy && best_tours && best_lens && ws, "NULL array argument");
        rc = choose_k(xy, offsets, B, &q, best_tours, best_lens, ws, ws_bytes, stream, q.k);
        if (rc != ACO_OK) return rc;
    }
    rc = aco_batch_setup(xy, offsets, B, &q, best_tours, best_lens, ws, ws_bytes, stream);
    if (rc != ACO_OK) return rc;
    BatchLayoutHost L;
    batch_layout(offsets, B, q.k, q.m, L);
    hipStream_t st = as_stream(stream);
    BatchState S = batch_state(ws, L, xy, B, q.k, q.m);
    int dev = 0;
    (void)hipGetDevice(&dev);
    const auto key = std::make_tuple(dev, q.k, q.m, L.nmax, B);
    Tuning best = default_tuning(q.k, L.nmax, q.m);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto f = g_tuned.find(key);
        if (f != g_tuned.end()) {
            best = f->second;
            autotune = 0;
        }
    }
    if (autotune && q.iterations > 0) {
        rc = tune_shape(S, L, &q, best_tours, best_lens, st, best);
        if (rc != ACO_OK) return rc;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[key] = best;
    }
    if (tuned_out) {
        tuned_out[0] = best.waves;
        tuned_out[1] = best.layout;
        tuned_out[2] = best.occ;
        tuned_out[3] = q.k;
    }
    if (q.iterations > 0) {
        rc = launch_colony(S, L, &q, 0, q.iterations, best, best_tours, best_lens, iter_best,
                           q.iterations, st);
        if (rc != ACO_OK) return rc;
    }
    return ACO_OK;
}
