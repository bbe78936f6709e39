// Per-ant tour construction and per-row choice weights, shared by the
// single-instance kernels and the batched persistent kernel.
#pragma once

#include "device.hpp"

namespace aco {

// Packed candidate row element: candidate city and its choice weight.
struct CandW {
    int32_t city;
    float w;
};

// Elements per choice row in memory: the scan width of k (the power of two
// the kernels are compiled for), at least 16, so that every row starts on a
// 128-byte line and a row of up to 16 candidates is one line (at k = 12 half
// the rows would otherwise straddle two lines).  A compile-time constant in
// the kernels (row_stride(KP) == row_stride(k)).
__host__ __device__ constexpr int row_stride(int k) { return k <= 16 ? 16 : k <= 32 ? 32 : 64; }

// Choice weights of one row, w[r] = tau^alpha * eta_b scaled by a per-row
// power of two (probabilities are invariant to a per-row factor).  For
// alpha in {0, 1} the value is the exact product rounded once to FP32 (times
// 2^E); for other alpha it is exp2(alpha log2 tau + log2 eta_b - row max).
struct SameCity {
    __device__ __forceinline__ int32_t operator()(int32_t c) const { return c; }
};

// The two forms of one element's unscaled weight: the product (alpha in
// {0, 1}) and its base-2 logarithm (other alpha; -inf for a zero factor).
__device__ __forceinline__ double choice_product(double alpha, float t, float eb)
{
    return (alpha == 1.0 ? (double)t : 1.0) * (double)eb;
}
__device__ __forceinline__ double choice_log2(double alpha, float t, float eb)
{
    const double td = (double)t, ed = (double)eb;
    return (td > 0.0 && ed > 0.0) ? alpha * log2(td) + log2(ed) : -INFINITY;
}

template <class CityMap = SameCity>
__device__ __forceinline__ void choice_row(const int32_t *__restrict__ nn,
                                           const float *__restrict__ tau,
                                           const float *__restrict__ eta_b, int k, double alpha,
                                           CandW *__restrict__ rows, CityMap map = CityMap())
{
    if (alpha == 1.0 || alpha == 0.0) {
        double mx = 0.0;
        for (int r = 0; r < k; ++r) {
            const double p = choice_product(alpha, tau[r], eta_b[r]);
            mx = p > mx ? p : mx;
        }
        const int e = (mx > 0.0) ? -ilogb(mx) : 0;
        for (int r = 0; r < k; ++r)
            rows[r] = CandW{map(nn[r]), (float)ldexp(choice_product(alpha, tau[r], eta_b[r]), e)};
    } else {
        double mx = -INFINITY;
        for (int r = 0; r < k; ++r) {
            const double lw = choice_log2(alpha, tau[r], eta_b[r]);
            mx = lw > mx ? lw : mx;
        }
        for (int r = 0; r < k; ++r) {
            const double lw = choice_log2(alpha, tau[r], eta_b[r]);
            rows[r] = CandW{map(nn[r]), (float)((mx > -INFINITY) ? exp2(lw - mx) : 0.0)};
        }
    }
}

// The same weights with one lane per element: the row's elements sit in an
// aligned group of KP lanes (KP a power of two >= k), lanes r >= k (act
// false) hold no element.  The row maximum is exact in any order, so the
// weights are those of choice_row bit for bit.  Every lane of the wave must
// call it (the maximum is taken with cross-lane moves).
template <int KP>
__device__ __forceinline__ float choice_weight_lane(bool act, float t, float eb, double alpha)
{
    if (alpha == 1.0 || alpha == 0.0) {
        const double p = act ? choice_product(alpha, t, eb) : 0.0;
        double mx = p;
#pragma unroll
        for (int off = KP / 2; off > 0; off >>= 1) {
            const double o = __shfl_xor(mx, off);
            mx = o > mx ? o : mx;
        }
        const int e = (mx > 0.0) ? -ilogb(mx) : 0;
        return (float)ldexp(p, e);
    }
    const double lw = act ? choice_log2(alpha, t, eb) : -INFINITY;
    double mx = lw;
#pragma unroll
    for (int off = KP / 2; off > 0; off >>= 1) {
        const double o = __shfl_xor(mx, off);
        mx = o > mx ? o : mx;
    }
    return (float)((mx > -INFINITY) ? exp2(lw - mx) : 0.0);
}

// Visited sets of one ant in LDS: one bit per city, or one byte per city
// (no read-modify-write; 8x the space).  Both are private to one wave, whose
// LDS operations complete in issue order.
struct VisBits {
    uint32_t *w;
    __device__ __forceinline__ static VisBits at(void *p) { return VisBits{(uint32_t *)p}; }
    __device__ __forceinline__ static size_t bytes(int64_t n) { return (size_t)((n + 31) / 32) * 4; }
    __device__ __forceinline__ uint32_t test(int c) const { return (w[c >> 5] >> (c & 31)) & 1u; }
    __device__ __forceinline__ void set(int c) const { atomicOr(&w[c >> 5], 1u << (c & 31)); }
    __device__ __forceinline__ void unset(int c) const
    {
        atomicAnd(&w[c >> 5], ~(1u << (c & 31)));
    }
    __device__ __forceinline__ void clear(int n, int lane) const
    {
        for (int i = lane; i < ((n + 31) >> 5); i += kWave) w[i] = 0u;
    }
    __device__ __forceinline__ void fill(int n, int lane) const
    {
        for (int i = lane; i < ((n + 31) >> 5); i += kWave) w[i] = ~0u;
    }
    // this lane's share of the count of marked cities (after clear and set)
    __device__ __forceinline__ int count(int n, int lane) const
    {
        int c = 0;
        for (int i = lane; i < ((n + 31) >> 5); i += kWave) c += __popc(w[i]);
        return c;
    }
};

struct VisBytes {
    uint8_t *b;
    __device__ __forceinline__ static VisBytes at(void *p) { return VisBytes{(uint8_t *)p}; }
    __device__ __forceinline__ static size_t bytes(int64_t n) { return (size_t)((n + 3) & ~3); }
    __device__ __forceinline__ uint32_t test(int c) const { return b[c]; }
    __device__ __forceinline__ void set(int c) const { b[c] = 1; }
    __device__ __forceinline__ void unset(int c) const { b[c] = 0; }
    __device__ __forceinline__ void clear(int n, int lane) const
    {
        uint32_t *w = (uint32_t *)b;
        for (int i = lane; i < ((n + 3) >> 2); i += kWave) w[i] = 0u;
    }
    __device__ __forceinline__ void fill(int n, int lane) const
    {
        uint32_t *w = (uint32_t *)b;
        for (int i = lane; i < ((n + 3) >> 2); i += kWave) w[i] = 0x01010101u;
    }
    __device__ __forceinline__ int count(int n, int lane) const
    {
        const uint32_t *w = (const uint32_t *)b;
        int c = 0;
        for (int i = lane; i < ((n + 3) >> 2); i += kWave) c += __popc(w[i] & 0x01010101u);
        return c;
    }
};

// A tour entry once resolved: the city index and its coordinates.
struct TourEntry {
    int32_t city;
    int2 p;
};

// The value of lane l - 1 (DPP wave shift right by one lane; lane 0's result
// is not used).
__device__ __forceinline__ int32_t from_prev_lane(int32_t v)
{
    return __builtin_amdgcn_update_dpp(v, v, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}

// How an ant names cities.  By index: the batched colonies.  By position in
// the grid's cell order: the single-instance construction, whose candidate
// rows, 64-NN table and visited set are all by position, so that the grid
// fallback can dismiss fully visited runs of cells with a few word reads.
// Tours are written as city indices in both.
struct CitySpace {
    static constexpr bool kLoad = false;   // a step's city index needs no load
    __device__ __forceinline__ int32_t from_city(const GridView &, int32_t c) const { return c; }
    __device__ __forceinline__ int32_t to_city(const GridView &, int32_t c) const { return c; }
    // city index of c and (kXY) its coordinates
    __device__ __forceinline__ int32_t city_xy(const GridView &, const int32_t *xy, int32_t c,
                                               int2 &p) const
    {
        p = ((const int2 *)xy)[c];
        return c;
    }
    template <bool kXY>
    __device__ __forceinline__ TourEntry fetch(const GridView &, const int32_t *xy, int32_t c) const
    {
        return TourEntry{c, kXY ? ((const int2 *)xy)[c] : make_int2(0, 0)};
    }
    template <class Vis, class Visited>
    __device__ __forceinline__ int32_t fallback(const GridView &g, const int32_t *xy, int32_t c,
                                                const Vis &, const Visited &visited) const
    {
        return fallback_city(g, xy, c, visited);
    }
};
struct PositionSpace {
    static constexpr bool kLoad = true;    // a position's city index is a load from pts
    __device__ __forceinline__ int32_t from_city(const GridView &g, int32_t c) const
    {
        return g.pinv[c];
    }
    __device__ __forceinline__ int32_t to_city(const GridView &g, int32_t q) const
    {
        return g.pts[q].z;
    }
    __device__ __forceinline__ int32_t city_xy(const GridView &g, const int32_t *, int32_t q,
                                               int2 &p) const
    {
        const int4 pt = g.pts[q];
        p = make_int2(pt.x, pt.y);
        return pt.z;
    }
    template <bool kXY>
    __device__ __forceinline__ TourEntry fetch(const GridView &g, const int32_t *, int32_t q) const
    {
        const int4 pt = g.pts[q];
        return TourEntry{pt.z, make_int2(pt.x, pt.y)};
    }
    template <class Visited>
    __device__ __forceinline__ int32_t fallback(const GridView &g, const int32_t *, int32_t c,
                                                const VisBits &vis, const Visited &) const
    {
        return fallback_position(g, c, VisitedByPosition{vis.w});
    }
};

struct AntTask {
    const int32_t *xy;     // [n][2]
    const CandW *rows;     // [n][row_stride(k)], rows and entries in the ant's city space
    int32_t n, k;
    uint32_t ant;          // absolute ant index (Philox counter word 1)
    uint32_t iteration;    // Philox counter word 2
    uint64_t seed;         // Philox key
    int32_t *tour;         // [n] output
    uint8_t *slots;        // [n] output
    float *prob;           // [n] output or nullptr
    // PartialACO (Section 3.1, Algorithm 1): the ant's local best tour (city
    // indices) or nullptr for a full construction; the partial-modification
    // threshold P = round(p 2^32) and the cap M on the rebuilt cities.
    const int32_t *lbest = nullptr;
    const int64_t *lbest_len = nullptr;   // this ant's local best length, or nullptr
    uint64_t p_threshold = 0;
    int32_t max_modify = 0;
    // Independent Roulette only: LDS for one block's uniforms, 64 steps x
    // ir_words_per_step(k) words (filled at the start of each block of steps)
    uint32_t *ir_words = nullptr;
    uint32_t *err = nullptr;   // the device's error word (guards), or nullptr
    uint64_t *prof = nullptr;  // step profile build only: kProfFields counters, or nullptr
};

// No closed tour is this long: every edge is shorter than 2^31 (coordinates
// within +-(2^29 - 1)), so a length of n * 2^31 or more is not a tour's.
__device__ __forceinline__ bool possible_tour_length(int64_t L, int32_t n)
{
    return L > 0 && L < ((int64_t)n << 31);
}

// Step profile (a separate build with ACO_STEP_PROFILE defined; the library
// itself is built without it).  Each ant's wave stamps the shader clock
// (s_memtime) at the points of every construction step where the row of the
// current city has arrived, its visited test is known, (roulette steps) the
// running sums' total is known, the next city is known, and the step ends
// (and once per block of 64 steps); the stamps are added up one step later,
// after the next visited test's LDS wait.  Fallback decisions are also
// counted by duration (a table chunk costs about one row load, a grid search
// several).  Per ant (kProfFields counters, lane 0 writes them at the end):
enum StepProfile {
    kProfTotal = 0,      // clock ticks of the whole build_ant call
    kProfRowWait = 1,    // end of the previous step (or block top) until the row of
                         // the current city has arrived
    kProfTail = 2,       // next city known until the end of the step (miss load
                         // issue, visited bit, staging)
    kProfBlock = 3,      // between blocks: Philox words, stores, tour entries
    kProfDecide = 4,     // visited test done until next city known, by path (+0..2):
                         // roulette scan, nearest-unvisited fallback,
                         // Independent Roulette
    kProfCount = 7,      // steps by the same paths (+0..2)
    kProfSteps = 10,     // steps
    kProfVisited = 11,   // row arrived until the visited test's ballot is known
    kProfFbMid = 12,     // fallback decisions of kFbMidTicks..kFbLongTicks: count, ticks (+1)
    kProfFbLong = 14,    // fallback decisions of kFbLongTicks or more: count, ticks (+1)
    kProfScan = 16,      // roulette steps: visited test done until the running sums'
                         // total is known (guess load issue, FP64 scan); the rest
                         // of the decision (draw, pick) stays in kProfDecide
    kProfFields = 18
};
constexpr uint64_t kFbMidTicks = 2000, kFbLongTicks = 6000;
#ifdef ACO_STEP_PROFILE
#define ACO_PROF(...) __VA_ARGS__
#else
#define ACO_PROF(...)
#endif

// The counters of one ant, held in scalar registers (no indexed array, which
// would live in scratch memory).
struct StepCounters {
    uint64_t total = 0, row = 0, tail = 0, block = 0, steps = 0, visited = 0, scan = 0;
    uint64_t dec[3] = {}, cnt[3] = {};
    __device__ __forceinline__ void decided(int path, uint64_t dt)
    {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            dec[p] += path == p ? dt : 0;
            cnt[p] += path == p ? 1 : 0;
        }
        ++steps;
    }
    // long fallback decisions go straight to the (zeroed) output, so that the
    // step loop carries no more registers; the store below leaves them alone
    __device__ __forceinline__ static void long_fallback(uint64_t *out, uint64_t dt)
    {
        if (!out || dt < kFbMidTicks) return;
        const int f = dt >= kFbLongTicks ? kProfFbLong : kProfFbMid;
        atomicAdd((unsigned long long *)&out[f], 1ull);
        atomicAdd((unsigned long long *)&out[f + 1], (unsigned long long)dt);
    }
    __device__ __forceinline__ void store(uint64_t *out) const
    {
        out[kProfTotal] = total;
        out[kProfRowWait] = row;
        out[kProfTail] = tail;
        out[kProfBlock] = block;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            out[kProfDecide + p] = dec[p];
            out[kProfCount + p] = cnt[p];
        }
        out[kProfSteps] = steps;
        out[kProfVisited] = visited;
        out[kProfScan] = scan;
    }
};

// Words of Independent Roulette uniforms held per step: k rounded up to the
// four words of a Philox block.
__host__ __device__ __forceinline__ int ir_words_per_step(int k) { return (k + 3) & ~3; }

// Builds one ant's tour with the whole wave (Section 2, Eq. 1).  Lane r < k
// holds candidate r of the current city.  The critical path of a step is:
// row load -> visited test (LDS) -> DPP scan -> ballot -> next row address.
// The row of the first candidate that can be chosen (the nearest; usually the
// heaviest) is loaded as soon as the visited test is done, so when the draw
// picks it the load overlaps the scan.  (Loading all k rows ahead costs more
// in loads and lane shuffles than the latency it hides.)  Steps run
// in blocks of 64: one Philox call gives the block's 64 words (lane l: step
// base + l) and the block's outputs are staged in lanes and stored together,
// so the inner loop holds only the step itself.
// KP is the scan width, the smallest power of two >= k.  `grid()` returns the
// instance's GridView (used by fallback steps).  With kLen the closed tour's
// length is summed on the way, exactly: each lane adds the edges that end at
// its staged steps (and at its share of a kept segment), one reduction at the
// end; otherwise 0 is returned.
template <int KP, bool kProb, int kSampler, bool kLen, class Space, class Vis, class GridFn>
__device__ int64_t build_ant_impl(const AntTask &T, const Vis &vis, const GridFn &grid,
                                  const Space &space)
{
    const int lane = lane_id();
    const int32_t n = T.n, k = T.k;
    auto visited = [&](int city) { return vis.test(city); };
    // (stamps of the previous step, added up once its results are known to
    // have arrived: after the next LDS wait, so that no wait is added)
    ACO_PROF(StepCounters pc; const uint64_t t_start = __builtin_amdgcn_s_memtime();
             uint64_t t_last = t_start, q0 = 0, q1 = 0, q1b = 0, q1c = 0, q2 = 0, q3 = 0;
             int qpath = -1;)

    const GridView g = grid();              // read once: no state carried through the loop
    uint32_t rnd = colony_draw(T.seed, T.iteration, T.ant, (uint32_t)lane);
    const uint32_t x0 = (uint32_t)read_lane_i32((int32_t)rnd, 0);
    const bool active = lane < k;
    const int lr = active ? lane : k - 1;   // idle lanes re-read a valid element
    const uint64_t act_mask = k >= kWave ? ~0ull : (1ull << k) - 1ull;   // lanes < k
    int64_t part = 0;                       // this lane's share of the tour length

    // PartialACO plan from words 0-2 of the block of step 0: keep the
    // lbest[s], ..., lbest[s + keep - 1] (cyclic) and rebuild n - keep cities
    int32_t keep = 0;
    int64_t s_pos = 0;
    if (T.lbest) {
        const uint4 plan = philox_block(0u, T.ant, T.iteration, 0u, (uint32_t)T.seed,
                                        (uint32_t)(T.seed >> 32));
        if ((uint64_t)plan.y < T.p_threshold) {
            const int64_t M = T.max_modify < 1 ? 1 : (T.max_modify > n - 1 ? n - 1 : T.max_modify);
            const int64_t r = 1 + (int64_t)(((uint64_t)plan.z * (uint64_t)M) >> 32);
            keep = (int32_t)(n - r);
            s_pos = (int64_t)(((uint64_t)plan.x * (uint64_t)n) >> 32);
        }
    }
    int32_t start, c;
    if (keep == 0) {
        vis.clear(n, lane);
        start = space.from_city(g, (int32_t)(((uint64_t)x0 * (uint64_t)n) >> 32));
        if (lane == 0) vis.set(start);
        c = start;
    } else {
        // the kept part is copied to the tour (no construction record: slot
        // kNoSlot); meanwhile the local best is checked to be a permutation:
        // its entries, marked by city index in the (cleared) bitmask, must
        // set n distinct bits.  A wrong row trips a guard (out-of-range
        // entries are read as city 0, so every access stays in range).
        // With its length given, that length must be a possible one, else the
        // kept part's length is summed edge by edge.
        const bool use_len =
            kLen && T.lbest_len && possible_tour_length(*T.lbest_len, n);
        if (kLen && T.lbest_len && !use_len && lane == 0) flag_error(T.err, kErrLbestLen);
        vis.clear(n, lane);
        bool row_ok = true;
        // copy eight positions per lane per round, loads issued before stores
        constexpr int kU = 8;
        int2 kprev = make_int2(0, 0);   // coordinates of kept position t0 - 1
        for (int32_t t0 = 0; t0 < keep; t0 += kU * kWave) {
            int32_t v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int32_t t = t0 + u * kWave + lane;
                int64_t q = s_pos + t;
                q -= q >= n ? n : 0;
                v[u] = t < keep ? T.lbest[q] : 0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int32_t t = t0 + u * kWave + lane;
                if (t < keep) {
                    const bool in = (uint32_t)v[u] < (uint32_t)n;
                    row_ok &= in;
                    v[u] = in ? v[u] : 0;
                    T.tour[t] = v[u];
                    T.slots[t] = (uint8_t)kNoSlot;
                    if constexpr (kProb) T.prob[t] = 1.0f;
                    vis.set(v[u]);
                }
            }
            if (kLen && !use_len) {
                int2 pc[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) pc[u] = ((const int2 *)T.xy)[v[u]];   // in range
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int32_t t = t0 + u * kWave + lane;
                    int2 prev = make_int2(from_prev_lane(pc[u].x), from_prev_lane(pc[u].y));
                    if (lane == 0) prev = kprev;
                    if (t >= 1 && t < keep)
                        part += nint_sqrt(sq_dist(prev.x, prev.y, pc[u].x, pc[u].y));
                    kprev.x = __builtin_amdgcn_readlane(pc[u].x, kWave - 1);
                    kprev.y = __builtin_amdgcn_readlane(pc[u].y, kWave - 1);
                }
            }
        }
        // the rebuilt part's entries complete the permutation check; then the
        // bitmask is set up for the construction (by the ant's city space):
        // every city visited except the n - keep to rebuild
        for (int32_t j = lane; j < n - keep; j += kWave) {
            const int32_t city = T.lbest[(s_pos + keep + j) % n];
            const bool in = (uint32_t)city < (uint32_t)n;
            row_ok &= in;
            vis.set(in ? city : 0);
        }
        int32_t marked = vis.count(n, lane);
        for (int off = kWave / 2; off > 0; off >>= 1) marked += __shfl_xor(marked, off);
        if (__builtin_amdgcn_ballot_w64(!row_ok) != 0ull || marked != n)
            if (lane == 0) flag_error(T.err, kErrLbestCity);
        vis.fill(n, lane);
        for (int32_t j = lane; j < n - keep; j += kWave) {
            const int32_t city = T.lbest[(s_pos + keep + j) % n];
            if ((uint32_t)city < (uint32_t)n) vis.unset(space.from_city(g, city));
        }
        if (kLen && use_len) {
            // the kept part's internal edges: the local best's length minus its
            // n - keep + 1 edges from the last kept city round to the first
            if (lane == 0) part += *T.lbest_len;
            for (int32_t u = lane; u <= n - keep; u += kWave) {
                int64_t q0 = s_pos + keep - 1 + u;   // < 2n - 1
                q0 -= q0 >= n ? n : 0;
                const int64_t q1 = q0 + 1 == n ? 0 : q0 + 1;
                const int32_t c0 = T.lbest[q0], c1 = T.lbest[q1];
                const int2 p0 = ((const int2 *)T.xy)[(uint32_t)c0 < (uint32_t)n ? c0 : 0];
                const int2 p1 = ((const int2 *)T.xy)[(uint32_t)c1 < (uint32_t)n ? c1 : 0];
                part -= nint_sqrt(sq_dist(p0.x, p0.y, p1.x, p1.y));
            }
        }
        const int32_t last_kept = T.lbest[(s_pos + keep - 1) % n];
        c = space.from_city(g, (uint32_t)last_kept < (uint32_t)n ? last_kept : 0);
        start = c;
    }
    const int32_t first = keep == 0 ? 1 : keep;   // first constructed tour position
    const int32_t store_from = keep;             // positions written by the step loop
    // coordinates of tour position first - 1 (the start or the last kept city)
    // and of position 0 (for the closing edge)
    int2 carry = make_int2(0, 0), head = make_int2(0, 0);
    if constexpr (kLen) {
        space.city_xy(g, T.xy, c, carry);
        head = carry;
        if (keep > 0) {
            const int32_t c0 = T.lbest[s_pos];
            head = ((const int2 *)T.xy)[(uint32_t)c0 < (uint32_t)n ? c0 : 0];
        }
    }

    // the previous block's tour entries, stored (and their edges summed) at
    // the end of the next block; lanes before the first stored step stand for
    // position first - 1 (coordinates `carry`)
    int32_t pend_city = 0, pend_x = 0, pend_y = 0;
    bool pend_mine = false, pend_any = false;
    int32_t pend_base = 0, pend_last = 0;
#define ACO_FLUSH_PENDING()                                                                    \
    do {                                                                                       \
        if (pend_mine) T.tour[pend_base + lane] = pend_city;                                  \
        if constexpr (kLen) {                                                                  \
            /* edge (t - 1, t) for every stored step t >= 1 */                                 \
            const int32_t px = pend_mine ? pend_x : carry.x, py = pend_mine ? pend_y : carry.y; \
            int32_t qx = from_prev_lane(px), qy = from_prev_lane(py);                         \
            if (lane == 0) {                                                                   \
                qx = carry.x;                                                                  \
                qy = carry.y;                                                                  \
            }                                                                                  \
            if (pend_mine && pend_base + lane >= 1) part += nint_sqrt(sq_dist(qx, qy, px, py)); \
            carry.x = __builtin_amdgcn_readlane(px, pend_last - pend_base);                    \
            carry.y = __builtin_amdgcn_readlane(py, pend_last - pend_base);                    \
        }                                                                                      \
    } while (0)
    // the next row is the guessed one (eg) or the one loaded after the draw
    // (en); the choice between them is made at the top of the next step, so
    // that a step whose guess missed issues its load before anything waits on
    // the guess
    constexpr int32_t ks = row_stride(KP);
    CandW eg = T.rows[(int64_t)c * ks + lr], en = eg;
    bool hit = true;
    bool next_bad = false;   // a next city came out of range (wave-uniform)
    for (int32_t base = first & ~(kWave - 1); base < n; base += kWave) {
        ACO_PROF(const uint64_t tb = __builtin_amdgcn_s_memtime(); pc.block += tb - t_last;
                 t_last = tb;)
        if (base > 0) rnd = colony_draw(T.seed, T.iteration, T.ant, (uint32_t)(base + lane));
        if constexpr (kSampler != 0) {
            // Independent Roulette: the block's uniforms, off the steps' critical
            // path; lane l computes step base + l, whose candidate r takes word
            // r mod 4 of the Philox block at counter (step, ant, iteration,
            // 1 + r / 4), and stores them at ir_words[l kw + r]
            const int kw = ir_words_per_step(k);
            for (int q = 0; q < kw / 4; ++q) {
                const uint4 blk = philox_block((uint32_t)(base + lane), T.ant, T.iteration,
                                               1u + (uint32_t)q, (uint32_t)T.seed,
                                               (uint32_t)(T.seed >> 32));
                *(uint4 *)&T.ir_words[lane * kw + 4 * q] = blk;
            }
        }
        // staged outputs: lane l holds step base + l (step 0 is the start city)
        int32_t st_city = start;
        uint32_t st_slot = kNoSlot;
        float st_prob = 1.0f;
        const int32_t last = min(base + kWave - 1, n - 1);
        for (int32_t step = max(base, first); step <= last; ++step) {
            const int idx = step - base;
            ACO_PROF(int path = 0;)
            const CandW e = hit ? eg : en;
            const int32_t j = e.city;
            ACO_PROF(asm volatile("" ::"s"(__builtin_amdgcn_readfirstlane(j)));
                     const uint64_t t1 = __builtin_amdgcn_s_memtime(); const uint64_t t0 = t_last;)
            const uint32_t seen = visited(j);          // every lane reads a valid word
            // Independent Roulette: this step's uniform for candidate lr (read
            // beside the visited word)
            const uint32_t xw = kSampler != 0 ? T.ir_words[idx * ir_words_per_step(k) + lr] : 0u;
            const bool live = active && seen == 0u && e.w > 0.0f;
            // the same lanes as ballot(live), from single-compare ballots (no
            // lane mask re-materialised in a vector register)
            const uint64_t any = __builtin_amdgcn_ballot_w64(seen == 0u) &
                                 __builtin_amdgcn_ballot_w64(e.w > 0.0f) & act_mask;
            ACO_PROF(asm volatile("" ::"s"(any)); const uint64_t t1b = __builtin_amdgcn_s_memtime();
                     uint64_t t1c = t1b; if (qpath >= 0) {
                pc.row += q1 - q0;
                pc.visited += q1b - q1;
                pc.scan += q1c - q1b;
                pc.decided(qpath, q2 - q1c);
                if (qpath == 1 && lane == 0) StepCounters::long_fallback(T.prof, q2 - q1b);
                pc.tail += q3 - q2;
            })
            // the first candidate that can be chosen is the likeliest next city
            // (rows are in distance order): its row is loaded while the scan runs
            // (issued without a branch: with no live candidate the row of lane
            // 63's valid city is loaded and serves only if that city is taken)
            const int32_t guess =
                read_lane_i32(j, __builtin_ctzll((unsigned long long)(any | (1ull << 63))));
            eg = T.rows[(int64_t)guess * ks + lr];
            const double wv = live ? (double)e.w : 0.0;
            int32_t jn;
            uint32_t slot;
            float prob = -1.0f;
            if constexpr (kSampler != 0) {
                // Independent Roulette: the largest product wins
                if (any) {
                    ACO_PROF(path = 2;)
                    const double v = live ? wv * ((double)xw * 0x1p-32) : -1.0;
                    const double vmax = read_lane_f64(wave_incl_max_f64(v, KP), k - 1);
                    const uint64_t top = __builtin_amdgcn_ballot_w64(v == vmax) & any;
                    const int f = __ffsll((unsigned long long)top) - 1;
                    jn = read_lane_i32(j, f);
                    slot = (uint32_t)f;
                } else {
                    ACO_PROF(path = 1;)
                    jn = space.fallback(g, T.xy, c, vis, visited);
                    slot = kNoSlot;
                }
            } else if (any) {
                // S > 0 exactly when some candidate is live (each live weight is
                // a positive FP32 value, so is their FP64 sum): the branch does
                // not wait for the scan, and u is formed while the scan runs
                const double u = (double)(uint32_t)read_lane_i32((int32_t)rnd, idx) * 0x1p-32;
                const double cum = wave_incl_scan_f64(wv, KP);
                const double S = read_lane_f64(cum, k - 1);
                ACO_PROF(asm volatile("" ::"s"(S)); t1c = __builtin_amdgcn_s_memtime();)
                const double target = u * S;
                const uint64_t hit = __builtin_amdgcn_ballot_w64(target < cum) & any;
                // first slot whose running sum passes the target; if rounding
                // leaves none, the last slot that can be chosen
                const int f = hit ? __ffsll((unsigned long long)hit) - 1
                                  : 63 - __clzll((long long)any);
                if constexpr (kProb) prob = (float)(read_lane_f64(wv, f) / S);
                jn = read_lane_i32(j, f);
                slot = (uint32_t)f;
            } else {
                ACO_PROF(path = 1;)
                jn = space.fallback(g, T.xy, c, vis, visited);
                slot = kNoSlot;
            }
            ACO_PROF(asm volatile("" ::"s"(jn)); const uint64_t t2 = __builtin_amdgcn_s_memtime();)
            // a city index is always in range here; the guard keeps a logic
            // error from turning into an out-of-bounds access (reported once
            // the tour is done, so the step stays branch-free and scalar)
            const bool out = (uint32_t)jn >= (uint32_t)n;
            next_bad |= out;
            jn = out ? start : jn;
            hit = jn == guess;
            if (!hit) en = T.rows[(int64_t)jn * ks + lr];
            if (lane == 0) vis.set(jn);
            if (lane == idx) {
                st_city = jn;
                st_slot = slot;
                if constexpr (kProb) st_prob = prob;
            }
            c = jn;
            ACO_PROF(const uint64_t t3 = __builtin_amdgcn_s_memtime(); t_last = t3; q0 = t0;
                     q1 = t1; q1b = t1b; q1c = t1c; q2 = t2; q3 = t3; qpath = path;)
        }
        // records go out now; the tour entries need a load (city index and
        // coordinates by position), so they go out one block later, when that
        // load has long arrived, instead of stalling the wave here
        const bool mine = base + lane <= last && base + lane >= store_from;
        if (mine) {
            T.slots[base + lane] = (uint8_t)st_slot;
            if constexpr (kProb) T.prob[base + lane] = st_prob;
        }
        if constexpr (!Space::kLoad && !kLen) {   // nothing to wait for
            if (mine) T.tour[base + lane] = st_city;
            continue;
        }
        if (pend_any) ACO_FLUSH_PENDING();
        if (mine) {
            const TourEntry te = space.template fetch<kLen>(g, T.xy, st_city);
            pend_city = te.city;
            pend_x = te.p.x;
            pend_y = te.p.y;
        }
        pend_mine = mine;
        pend_base = base;
        pend_last = last;
        pend_any = true;
    }
    if (pend_any) ACO_FLUSH_PENDING();
#undef ACO_FLUSH_PENDING
    if (next_bad && lane == 0) flag_error(T.err, kErrNextCity);
    ACO_PROF(if (qpath >= 0) {
        pc.row += q1 - q0;
        pc.visited += q1b - q1;
        pc.scan += q1c - q1b;
        pc.decided(qpath, q2 - q1c);
        pc.tail += q3 - q2;
    } if (T.prof && lane == 0) {
        pc.total = __builtin_amdgcn_s_memtime() - t_start;
        pc.store(T.prof);
    })
    if constexpr (!kLen) return 0;
    // the closing edge (position n - 1 to position 0), then one reduction
    if (lane == 0) part += nint_sqrt(sq_dist(carry.x, carry.y, head.x, head.y));
    for (int off = kWave / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
    // a local best length that does not match its row can leave the sum at a
    // length no tour has
    if (keep > 0 && !possible_tour_length(part, n) && lane == 0) flag_error(T.err, kErrLbestLen);
    return part;
}

// kSampler selects the next-city rule at compile time, so each kernel holds
// one of them only: 0 the roulette of Eq. 1; 1 Independent Roulette (Section
// 3: the largest w_r U_r, U_r from word r mod 4 of the Philox block at
// counter (t, ant, iteration, 1 + r / 4), ties to the lower rank).
template <int KP, class Space = CitySpace, int kSampler = 0, bool kLen = false, class Vis,
          class GridFn>
__device__ int64_t build_ant(const AntTask &T, const Vis &vis, const GridFn &grid,
                             const Space &space = Space())
{
    if (T.prob)
        return build_ant_impl<KP, true, kSampler, kLen>(T, vis, grid, space);
    else
        return build_ant_impl<KP, false, kSampler, kLen>(T, vis, grid, space);
}

// The same with the probability record fixed at compile time (kProb: T.prob
// is written; otherwise it is ignored), for kernels that hold one variant only.
template <int KP, bool kProb, class Space, int kSampler, bool kLen, class Vis, class GridFn>
__device__ int64_t build_ant_fixed(const AntTask &T, const Vis &vis, const GridFn &grid,
                                   const Space &space = Space())
{
    return build_ant_impl<KP, kProb, kSampler, kLen>(T, vis, grid, space);
}

// The kx nearest cities of city `me` in (d, index) order, by one thread:
// square blocks of cells of growing radius (1, 3, 7, ...), a sorted list of
// keys (d << 32 | city) in LDS at L[0], L[ls], L[2 ls], ...; the search stops
// once every point outside the searched block is farther than the kx-th
// distance.  Requires kx <= (number of other cities).
__device__ inline void knn_city(const GridView &g, const int4 me, int kx, uint64_t *L, int ls)
{
    const GridHdr &h = g.h;
    const int gx = cell_x(h, me.x), gy = cell_y(h, me.y);
    int cnt = 0;
    int rin = -1;
    for (int r = 1;; rin = r, r = 2 * r + 1) {
        const int nslots = 2 * (2 * r + 1);
        for (int s = 0; s < nslots; ++s) {
            int row, xa, xb;
            if (!block_slot(h, gx, gy, rin, r, s, row, xa, xb)) continue;
            const int a = g.cell_start[(int64_t)row * h.gw + xa];
            const int b = g.cell_start[(int64_t)row * h.gw + xb + 1];
            for (int q = a; q < b; ++q) {
                const int4 pt = g.pts[q];
                if (pt.z == me.z) continue;
                const uint64_t key =
                    ((uint64_t)(uint32_t)nint_sqrt(sq_dist(me.x, me.y, pt.x, pt.y)) << 32) |
                    (uint32_t)pt.z;
                if (cnt == kx && key >= L[(int64_t)(kx - 1) * ls]) continue;
                int pos = cnt < kx ? cnt++ : kx - 1;
                while (pos > 0 && L[(int64_t)(pos - 1) * ls] > key) {
                    L[(int64_t)pos * ls] = L[(int64_t)(pos - 1) * ls];
                    --pos;
                }
                L[(int64_t)pos * ls] = key;
            }
        }
        int64_t bound;
        if (!outside_bound(h, me.x, me.y, gx, gy, r, bound)) break;
        if (cnt == kx && bound > (int64_t)(L[(int64_t)(kx - 1) * ls] >> 32)) break;
    }
}

// The same list for a wide table (hundreds of entries), by one thread: a
// max-heap of the kx smallest keys in LDS at L[0], L[ls], ... (O(log kx) per
// kept point instead of a shift of the sorted list), rings of cells one radius
// at a time (the doubling blocks above would read many more points than a
// wide list needs), the same stopping rule against the heap's root, and a heap
// sort into (d, index) order at the end.  Requires kx <= (number of other
// cities).
__device__ inline void knn_heap_down(uint64_t *L, int ls, int cnt, int i, uint64_t key)
{
    for (;;) {
        int c = 2 * i + 1;
        if (c >= cnt) break;
        uint64_t cv = L[(int64_t)c * ls];
        if (c + 1 < cnt) {
            const uint64_t c2 = L[(int64_t)(c + 1) * ls];
            if (c2 > cv) {
                cv = c2;
                ++c;
            }
        }
        if (cv <= key) break;
        L[(int64_t)i * ls] = cv;
        i = c;
    }
    L[(int64_t)i * ls] = key;
}

__device__ inline void knn_city_wide(const GridView &g, const int4 me, int kx, uint64_t *L, int ls)
{
    const GridHdr &h = g.h;
    const int gx = cell_x(h, me.x), gy = cell_y(h, me.y);
    int cnt = 0;
    for (int r = 1, rin = -1;; rin = r, ++r) {
        const int nslots = 2 * (2 * r + 1);
        for (int s = 0; s < nslots; ++s) {
            int row, xa, xb;
            if (!block_slot(h, gx, gy, rin, r, s, row, xa, xb)) continue;
            const int a = g.cell_start[(int64_t)row * h.gw + xa];
            const int b = g.cell_start[(int64_t)row * h.gw + xb + 1];
            for (int q = a; q < b; ++q) {
                const int4 pt = g.pts[q];
                if (pt.z == me.z) continue;
                const uint64_t key =
                    ((uint64_t)(uint32_t)nint_sqrt(sq_dist(me.x, me.y, pt.x, pt.y)) << 32) |
                    (uint32_t)pt.z;
                if (cnt < kx) {
                    int i = cnt++;   // sift up
                    while (i > 0) {
                        const int pi = (i - 1) >> 1;
                        const uint64_t pv = L[(int64_t)pi * ls];
                        if (pv >= key) break;
                        L[(int64_t)i * ls] = pv;
                        i = pi;
                    }
                    L[(int64_t)i * ls] = key;
                } else if (key < L[0]) {
                    knn_heap_down(L, ls, kx, 0, key);
                }
            }
        }
        int64_t bound;
        if (!outside_bound(h, me.x, me.y, gx, gy, r, bound)) break;
        if (cnt == kx && bound > (int64_t)(L[0] >> 32)) break;
    }
    for (int end = cnt - 1; end > 0; --end) {   // heap sort: ascending keys
        const uint64_t top = L[0], last = L[(int64_t)end * ls];
        L[(int64_t)end * ls] = top;
        knn_heap_down(L, ls, end, 0, last);
    }
}

// The nearest-neighbour tour from city 0 by one wave: the first unvisited
// candidate of the current city when there is one (candidate keys are smaller
// than all others), else the nearest unvisited city (64-NN table, then grid).
// Writes the tour and returns its closed length.
template <class Vis>
__device__ int64_t nn_tour_wave(const int32_t *__restrict__ xy, int32_t n, int32_t k,
                                const int32_t *__restrict__ nn, const int32_t *__restrict__ nnd,
                                const GridView &g, const Vis &vis, int32_t *tour,
                                uint32_t *err = nullptr)
{
    const int lane = lane_id();
    vis.clear(n, lane);
    auto visited = [&](int city) { return vis.test(city); };
    if (lane == 0) vis.set(0);
    int32_t c = 0;
    int64_t L = 0;
    int32_t stage = 0;   // lane t holds tour[base + t]
    bool next_bad = false;
    for (int32_t t = 1; t < n; ++t) {
        const int64_t rb = (int64_t)c * k;
        int32_t j = 0, d = 0;
        bool unv = false;
        if (lane < k) {
            j = nn[rb + lane];
            d = nnd[rb + lane];
            unv = !visited(j);
        }
        const uint64_t bal = __ballot(unv);
        int32_t jn, dn;
        if (bal) {
            const int f = __ffsll((unsigned long long)bal) - 1;
            jn = read_lane_i32(j, f);
            dn = read_lane_i32(d, f);
        } else {
            jn = fallback_city(g, xy, c, visited);
            const bool out = (uint32_t)jn >= (uint32_t)n;   // range guard, as in build_ant
            next_bad |= out;
            jn = out ? 0 : jn;
            dn = nint_sqrt(sq_dist(xy[2 * (int64_t)c], xy[2 * (int64_t)c + 1],
                                   xy[2 * (int64_t)jn], xy[2 * (int64_t)jn + 1]));
        }
        if (lane == 0) vis.set(jn);
        if (lane == (t & 63)) stage = jn;
        if ((t & 63) == 63 || t == n - 1) {
            const int32_t base = t & ~63;
            if (base + lane <= t) tour[base + lane] = stage;
        }
        L += dn;
        c = jn;
    }
    L += nint_sqrt(sq_dist(xy[2 * (int64_t)c], xy[2 * (int64_t)c + 1], xy[0], xy[1]));
    if (next_bad && lane == 0) flag_error(err, kErrNextCity);
    return L;
}

// Rows of the two-hop table by position: row c holds, in four groups of 16
// entries, the first 16 entries of c's neighbour row and of the rows of its
// three nearest neighbours (-1 where a row is shorter or absent).
constexpr int kHopGroups = 4, kHopWidth = 16 * kHopGroups;

// The nearest-neighbour tour from city 0 by one wave, on positions: the
// nearest unvisited city is the first unvisited entry of the current city's
// neighbour row (the candidate list is its prefix, in the same order; the
// first 16 entries settle most steps), else the grid's nearest unvisited city
// (fallback_position).  Writes the tour as city indices; its length is summed
// afterwards, off this sequential loop.  Two steps per row load where it
// can: the two-hop row of c also holds the rows of c's three nearest
// neighbours, so when the step from c goes to one of them (the usual case)
// the next step is decided from the same load.  Every entry is tested against
// the visited set as it stands before the first of the two steps; the city
// the first step takes is not in its own row, so the second step sees what it
// would have seen after a load of its own row.
__device__ inline void nn_tour_positions_hop(const GridView &g, int32_t n, const VisBits &vis,
                                             const int32_t *__restrict__ hop, int32_t *tour,
                                             uint32_t *err = nullptr)
{
    const int lane = lane_id();
    vis.clear(n, lane);
    const VisitedByPositionAfterLoad vp{{vis.w}};
    int32_t c = g.pinv[0];
    if (lane == 0) vis.set(c);
    int32_t stage = c;   // lane t holds the position of tour[base + t]
    bool next_bad = false;
    int32_t t = 1;
    auto take = [&](int32_t jn) {   // step t goes to jn
        const bool out = (uint32_t)jn >= (uint32_t)n;   // range guard, as in build_ant
        next_bad |= out;
        jn = out ? c : jn;
        if (lane == 0) vis.set(jn);
        if (lane == (t & 63)) stage = jn;
        if ((t & 63) == 63 || t == n - 1) {
            const int32_t base = t & ~63;
            if (base + lane <= t) tour[base + lane] = g.pts[stage].z;
        }
        c = jn;
        ++t;
    };
    while (t < n) {
        const int32_t h = hop[(int64_t)c * kHopWidth + lane];
        const uint64_t bal = __ballot(h >= 0 && !vis.test(h));
        const uint64_t b0 = bal & 0xFFFFull;
        const int f = b0 ? __ffsll((unsigned long long)b0) - 1 : kWave;
        take(b0 ? read_lane_i32(h, f) : fallback_position(g, c, vp));
        if (f < kHopGroups - 1 && t < n) {
            // the row of the city just taken is group f + 1 of this load
            const uint64_t b1 = (bal >> (16 * (f + 1))) & 0xFFFFull;
            take(b1 ? read_lane_i32(h, 16 * (f + 1) + __ffsll((unsigned long long)b1) - 1)
                    : fallback_position(g, c, vp));
        }
    }
    if (next_bad && lane == 0) flag_error(err, kErrNextCity);
}

}  // namespace aco
