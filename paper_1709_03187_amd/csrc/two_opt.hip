// Windowed 2-opt local search (2-opt with a small probability, Section 4;
// moves limited to edges within W tour positions, Section 5).
//
// Rounds of non-overlapping best moves, so that one round applies many moves
// at once.  Per round and tour:
//   k_two_opt_eval    one thread per position i evaluates its W' - 1 moves
//                     from an LDS tile of the coordinates of positions
//                     i0 .. i0 + 256 + W' + 1 and keeps the best as one int64
//                     key g * 2^12 + o (g < 0), or kNone;
//   k_two_opt_accept  a position's move is taken when no move whose span
//                     meets its own is better by (g, position), read from an
//                     LDS tile of keys i0 - W' - 1 .. i0 + 256 + W';
//   k_two_opt_apply   one wave per taken move reverses t[i+1 .. i+o], marks
//                     the changed construction records and the tiles whose
//                     keys read a changed position.
// Only tiles marked by the previous round are evaluated again: a key depends
// on positions i .. i + W' + 1 alone, so the others are still exact.  All
// distances are integers and all sums exact, so the result does not depend
// on scheduling.
#include <cmath>

#include "common.hpp"
#include "device.hpp"

namespace aco {
namespace {

constexpr int kT = 256;                 // positions per workgroup
constexpr int kOffBits = 12;            // offset field of a key (W <= 2048 < 4096)
constexpr int64_t kOffMask = (1 << kOffBits) - 1;
constexpr int64_t kNone = INT64_MAX;    // no improving move
constexpr int kRoundsPerSync = 16;      // rounds launched between host reads
constexpr int kApplyBlocks = 256;

__device__ __forceinline__ int64_t d_int(int2 p, int2 q)
{
    return nint_sqrt(sq_dist(p.x, p.y, q.x, q.y));
}

// nint(sqrt(dx^2 + dy^2)) for |dx|, |dy| < 2^21, exactly, without 64-bit
// integer products: s < 2^43 is exact in FP64; the FP32 root of fl32(s) is
// within 2^-22.7 relative, i.e. < 0.45 absolute, of sqrt(s) (below 2^21.5), so
// k = rint(root) is nint(sqrt(s)) or one off.  With t = s - k^2 (exact):
// sqrt(s) >= k + 1/2 iff t > k, and sqrt(s) < k - 1/2 iff t <= -k for k >= 1
// (sqrt(s) is never a half-integer; k = 0 only for s = 0).
__device__ __forceinline__ int32_t d_small(int2 p, int2 q)
{
    const double dx = (double)(p.x - q.x), dy = (double)(p.y - q.y);
    const double s = __builtin_fma(dx, dx, dy * dy);
    const float kf = __builtin_rintf(__builtin_amdgcn_sqrtf((float)s));   // v_sqrt_f32, 1 ulp
    const double k = (double)kf;
    const double t = __builtin_fma(-k, k, s);
    return (int32_t)kf + (t > k ? 1 : 0) - ((kf > 0.0f && t <= -k) ? 1 : 0);
}

// Evaluation tiles: each wave covers 63 positions; its lane l computes
// D_o(q) = d(t_q, t_q+o) for q = its position, and the gain of move (q, o)
// takes D_o(q + 1) from lane l + 1 (so lane 63 only supplies that distance):
//   g(q, o) = D_o(q) + D_o(q + 1) - L[q] - L[q + o].
constexpr int kPosPerWave = kWave - 1;
constexpr int kTE = (kT / kWave) * kPosPerWave;   // 252 positions per evaluation tile

// The value of lane l + 1 (DPP wave shift by one lane; lane 63 receives 0).
__device__ __forceinline__ int32_t from_next_lane(int32_t v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}

// Best key of tile position q (lanes 63 return garbage, unused).
template <bool kSmall>
__device__ __forceinline__ int64_t best_move(const int2 *P, const int32_t *L, int32_t q,
                                             int32_t W)
{
    const int2 a = P[q];
    const int32_t lq = L[q];
    if constexpr (kSmall) {
        // distances below 2^21.5: gains fit in int32
        int32_t bg = 0, bo = 0;
        for (int32_t o = 2; o <= W; ++o) {
            const int32_t dq = d_small(a, P[q + o]);
            const int32_t dq1 = from_next_lane(dq);
            const int32_t g = dq + dq1 - lq - L[q + o];
            bo = g < bg ? o : bo;          // strict: the smaller offset keeps a tie
            bg = g < bg ? g : bg;
        }
        return bg < 0 ? (int64_t)bg * (1 << kOffBits) + bo : kNone;
    } else {
        int64_t bg = 0;
        int32_t bo = 0;
        for (int32_t o = 2; o <= W; ++o) {
            const int32_t dq = (int32_t)d_int(a, P[q + o]);   // < 2^31 for |coords| < 2^29
            const int32_t dq1 = from_next_lane(dq);
            const int64_t g = (int64_t)dq + dq1 - lq - L[q + o];
            bo = g < bg ? o : bo;
            bg = g < bg ? g : bg;
        }
        return bg < 0 ? bg * (1 << kOffBits) + bo : kNone;
    }
}

template <bool kSmall>
__device__ __forceinline__ int64_t dist_t(int2 p, int2 q)
{
    if constexpr (kSmall)
        return d_small(p, q);
    else
        return d_int(p, q);
}

__device__ __forceinline__ int64_t move_key(int64_t g, int32_t o)
{
    return g < 0 ? g * (1 << kOffBits) + o : kNone;
}

// Every move of one position qf by the whole wave (lane l takes offsets
// 2 + l, 2 + l + 64, ...), reduced to the wave's minimum key.
template <bool kSmall>
__device__ __forceinline__ int64_t one_position(const int2 *P, const int32_t *L, int32_t qf,
                                                int32_t W, int lane)
{
    const int2 a = P[qf], b = P[qf + 1];
    const int64_t lq = L[qf];
    int64_t best = kNone;
    for (int32_t o = 2 + lane; o <= W; o += kWave) {
        const int64_t k = move_key(dist_t<kSmall>(a, P[qf + o]) + dist_t<kSmall>(b, P[qf + o + 1]) -
                                       lq - L[qf + o],
                                   o);
        best = k < best ? k : best;
    }
    // signed order through the unsigned DPP minimum: flip the sign bit
    return (int64_t)(wave_min_u64_dpp((uint64_t)best ^ (1ull << 63)) ^ (1ull << 63));
}

// The moves of position q whose far edge changed: x = q + o in the wave's list
// of positions with C2[x] set, folded into `best` (the kept key).
template <bool kSmall>
__device__ __forceinline__ int64_t changed_moves(const int2 *P, const int32_t *L,
                                                 const int16_t *list, int32_t cnt, int32_t q,
                                                 int32_t W, int64_t best)
{
    const int2 a = P[q], b = P[q + 1];
    const int64_t lq = L[q];
    for (int32_t e = 0; e < cnt; ++e) {
        const int32_t x = list[e];
        const int32_t o = x - q;
        if (o >= 2 && o <= W) {
            const int64_t k =
                move_key(dist_t<kSmall>(a, P[x]) + dist_t<kSmall>(b, P[x + 1]) - lq - L[x], o);
            best = k < best ? k : best;
        }
    }
    return best;
}

// Participating ants, in increasing order: one workgroup, wave ballots.
__global__ __launch_bounds__(kT) void k_two_opt_select(uint64_t seed, uint32_t iteration,
                                                       int32_t m, uint64_t thr, int32_t *sel,
                                                       int32_t *count, int64_t *gain_sum)
{
    __shared__ int32_t wsum[kT / kWave];
    __shared__ int32_t base;
    const int lane = lane_id(), w = threadIdx.x / kWave;
    if (threadIdx.x == 0) {
        base = 0;
        *gain_sum = 0;
    }
    __syncthreads();
    for (int32_t a0 = 0; a0 < m; a0 += kT) {
        const int32_t a = a0 + (int32_t)threadIdx.x;
        bool take = false;
        if (a < m) {
            const uint4 b = philox_block(0u, (uint32_t)a, iteration, 0u, (uint32_t)seed,
                                         (uint32_t)(seed >> 32));
            take = (uint64_t)b.w < thr;
        }
        const uint64_t bal = __builtin_amdgcn_ballot_w64(take);
        if (lane == 0) wsum[w] = __popcll(bal);
        __syncthreads();
        int32_t off = base;
        for (int q = 0; q < w; ++q) off += wsum[q];
        if (take) sel[off + __popcll(bal & ((1ull << lane) - 1ull))] = a;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int q = 0; q < kT / kWave; ++q) base += wsum[q];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base;
}

// Dirty flags: buffer 0 all set (round 0 evaluates every tile), buffer 1
// clear; change stamps of the S tours' positions: never changed.
__global__ void k_two_opt_init(uint32_t *dirty, int32_t tiles, int32_t batch, int32_t S,
                               int32_t *stamp, int64_t stamps)
{
    const int64_t per = (int64_t)S * tiles;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < per;
         q += (int64_t)gridDim.x * blockDim.x) {
        dirty[q] = 1u;
        dirty[(int64_t)batch * tiles + q] = 0u;
    }
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < stamps;
         q += (int64_t)gridDim.x * blockDim.x)
        stamp[q] = -2;
}

// Coordinates in tour order of the S tours: pxy[s][p] = xy[tours[ants[s]][p]].
__global__ void k_two_opt_coords(const int32_t *__restrict__ xy, const int32_t *__restrict__ tours,
                                 const int32_t *__restrict__ ants, int32_t n, int32_t S,
                                 int2 *__restrict__ pxy)
{
    const int64_t total = (int64_t)S * n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = q / n, p = q - s * n;
        const int32_t c = tours[(int64_t)ants[s] * n + p];
        pxy[q] = ((const int2 *)xy)[(uint32_t)c < (uint32_t)n ? c : 0];   // tours are permutations
    }
}

__global__ void k_two_opt_zero(int32_t *p, int32_t count)
{
    for (int32_t q = threadIdx.x; q < count; q += blockDim.x) p[q] = 0;
}

// Best move of every position of the dirty tiles.  Grid (tiles, S).
//
// Round 0 evaluates every move.  Later rounds know which positions the
// previous round changed (stamp == round - 1): a move's gain depends only on
// the cities at positions q, q + 1, q + o, q + o + 1, so with C2[x] = "x or
// x + 1 changed" a position q is re-evaluated in full when C2[q] (its own
// edge) or C2[q + o_best] (its kept best move) is set, and otherwise only its
// moves with C2[q + o] set are recomputed and folded into the kept key.  Full
// positions are done one at a time by the whole wave.  A wave runs every
// move of all its lanes instead (round 0, or when that is cheaper): that costs
// W' distances per lane, the other way 2 per listed position plus
// 2 ceil((W' - 1) / 64) per full position.

template <bool kSmall>
__device__ __forceinline__ int64_t eval_wave(const int2 *P, const int32_t *L, const uint8_t *C2,
                                             int16_t *list, int32_t q0, int lane, int32_t W,
                                             bool first, bool valid, int64_t old)
{
    const int32_t q = q0 + lane;
    const bool full = first || (valid && (C2[q] || (old != kNone && C2[q + (int32_t)(old & kOffMask)])));
    const uint64_t fmask = __builtin_amdgcn_ballot_w64(full && valid);
    if (first) return best_move<kSmall>(P, L, q, W);
    // positions x = q0 + 2 .. q0 + 62 + W with C2[x] set, in order
    int32_t cnt = 0;
    for (int32_t x0 = q0 + 2; x0 <= q0 + kPosPerWave - 1 + W; x0 += kWave) {
        const int32_t x = x0 + lane;
        const bool c = x <= q0 + kPosPerWave - 1 + W && C2[x];
        const uint64_t bal = __builtin_amdgcn_ballot_w64(c);
        if (c) list[cnt + __popcll(bal & ((1ull << lane) - 1ull))] = (int16_t)x;
        cnt += __popcll(bal);
    }
    __builtin_amdgcn_wave_barrier();
    const int32_t per_full = 2 * ((W - 2) / kWave + 1);
    if (2 * cnt + __popcll(fmask) * per_full >= W) return best_move<kSmall>(P, L, q, W);
    int64_t key = changed_moves<kSmall>(P, L, list, cnt, q, W, full ? kNone : old);
    for (uint64_t f = fmask; f; f &= f - 1) {
        const int fl = __ffsll((unsigned long long)f) - 1;
        const int64_t k = one_position<kSmall>(P, L, q0 + fl, W, lane);
        key = lane == fl ? k : key;
    }
    return key;
}

__global__ __launch_bounds__(kT) void k_two_opt_eval(const int2 *__restrict__ pxy, int32_t n,
                                                     int32_t W, int32_t tiles, int32_t round,
                                                     const int32_t *__restrict__ stamp,
                                                     uint32_t *__restrict__ dirty_cur,
                                                     int64_t *__restrict__ keys,
                                                     int32_t *__restrict__ list_count)
{
    // LDS: P int2 [np] (coordinates of positions i0 .. i0 + kTE + W + 1),
    // L int32 [np], per-wave lists int16 [4][kPosPerWave + W], C2 uint8 [np],
    // CH uint8 [np] (position changed in the previous round)
    extern __shared__ int2 P[];
    __shared__ uint32_t go;
    __shared__ int32_t box[4];    // min x, max x, min y, max y of the tile
    const int32_t s = blockIdx.y, tile = blockIdx.x;
    if (threadIdx.x == 0) {
        if (tile == 0) list_count[s] = 0;   // the previous round's list is consumed
        uint32_t *flag = dirty_cur + (int64_t)s * tiles + tile;
        go = *flag;
        if (go) *flag = 0u;
        box[0] = box[2] = INT32_MAX;
        box[1] = box[3] = INT32_MIN;
    }
    __syncthreads();
    if (!go) return;
    const int32_t np = kTE + W + 2;
    int32_t *L = (int32_t *)(P + np);     // L[q] = d(P[q], P[q + 1])
    int16_t *lists = (int16_t *)(L + np);
    uint8_t *C2 = (uint8_t *)(lists + (kT / kWave) * (kPosPerWave + W));
    uint8_t *CH = C2 + np;
    const int2 *pc = pxy + (int64_t)s * n;   // coordinates in tour order
    const int32_t *st = stamp + (int64_t)s * n;
    const int32_t i0 = tile * kTE;
    const bool first = round == 0;
    int32_t x0 = INT32_MAX, x1 = INT32_MIN, y0 = INT32_MAX, y1 = INT32_MIN;
    for (int32_t q = threadIdx.x; q < np; q += kT) {
        int64_t pos = (int64_t)i0 + q;
        pos -= pos >= n ? n : 0;
        pos = pos >= n ? pos % n : pos;   // tiles longer than the tour wrap again
        const int2 pt = pc[pos];
        P[q] = pt;
        x0 = min(x0, pt.x);
        x1 = max(x1, pt.x);
        y0 = min(y0, pt.y);
        y1 = max(y1, pt.y);
        if (!first) CH[q] = st[pos] == round - 1 ? 1 : 0;
    }
    atomicMin(&box[0], x0);
    atomicMax(&box[1], x1);
    atomicMin(&box[2], y0);
    atomicMax(&box[3], y1);
    __syncthreads();
    // coordinates spanning less than 2^21 in both axes make every difference small
    const bool small = (int64_t)box[1] - box[0] < (1 << 21) && (int64_t)box[3] - box[2] < (1 << 21);
    for (int32_t q = threadIdx.x; q < np - 1; q += kT) {
        L[q] = small ? d_small(P[q], P[q + 1]) : (int32_t)d_int(P[q], P[q + 1]);
        if (!first) C2[q] = CH[q] | CH[q + 1];
    }
    __syncthreads();
    // whole waves run the loops (lane l + 1 feeds lane l)
    const int lane = lane_id();
    const int32_t w = (int32_t)(threadIdx.x / kWave);
    const int32_t q0 = w * kPosPerWave, i = i0 + q0 + lane;
    const bool valid = lane < kPosPerWave && i < n;
    const int64_t old = (!first && valid) ? keys[(int64_t)s * n + i] : kNone;
    int16_t *list = lists + w * (kPosPerWave + W);
    const int64_t key = small ? eval_wave<true>(P, L, C2, list, q0, lane, W, first, valid, old)
                              : eval_wave<false>(P, L, C2, list, q0, lane, W, first, valid, old);
    if (valid) keys[(int64_t)s * n + i] = key;
}

// A position's move is taken when no overlapping move is better by (g, position).
// Grid (ceil(n / kT), S).  Each wave takes the candidates among its 64
// positions one at a time and checks the moves that can overlap with all
// lanes, nearest first, 64 at a time, stopping at the first better one: moves
// starting inside the span (d = 1 .. o + 1 ahead; they always overlap), then
// moves starting d = 1 .. W + 1 before it (they overlap when o_u + 1 >= d).
__global__ __launch_bounds__(kT) void k_two_opt_accept(const int64_t *__restrict__ keys,
                                                       int32_t n, int32_t W,
                                                       int32_t *__restrict__ list,
                                                       int32_t list_cap,
                                                       int32_t *__restrict__ list_count,
                                                       int32_t *__restrict__ round_moves)
{
    extern __shared__ int64_t K[];   // keys of positions i0 - W - 1 .. i0 + kT + W
    const int32_t s = blockIdx.y, i0 = blockIdx.x * kT, t = threadIdx.x, i = i0 + t;
    const int64_t *ks = keys + (int64_t)s * n;
    const int64_t mine = i < n ? ks[i] : kNone;
    if (!__syncthreads_or(mine != kNone)) return;
    const int32_t nk = kT + 2 * W + 2;
    for (int32_t q = t; q < nk; q += kT) {
        int64_t pos = ((int64_t)i0 - W - 1 + q) % n;
        pos += pos < 0 ? n : 0;
        K[q] = ks[pos];
    }
    __syncthreads();
    const int lane = lane_id();
    const int32_t w0 = (int32_t)(t / kWave) * kWave;   // first tile position of this wave
    uint64_t cand = __builtin_amdgcn_ballot_w64(mine != kNone);
    while (cand) {
        const int32_t tc = w0 + __ffsll((unsigned long long)cand) - 1;
        cand &= cand - 1;
        const int32_t ic = i0 + tc;                    // < n: only real positions have keys
        const int64_t kc = K[tc + W + 1];
        const int64_t gc = kc >> kOffBits;
        const int32_t oc = (int32_t)(kc & kOffMask);
        const int32_t span = (oc + 1) + (W + 1);
        bool better = false;
        for (int32_t j0 = 0; j0 < span && !better; j0 += kWave) {
            const int32_t j = j0 + lane;
            bool b = false;
            if (j < span) {
                const bool ahead = j <= oc;
                const int32_t d = ahead ? j + 1 : oc - j;   // ahead: 1 .. o + 1; behind: -1 .. -(W + 1)
                const int64_t ku = K[tc + W + 1 + d];
                if (ku != kNone && (ahead || (int32_t)(ku & kOffMask) + 1 >= -d)) {
                    int32_t u = ic + d;                    // W + 1 < n: one wrap at most
                    u += u < 0 ? n : 0;
                    u -= u >= n ? n : 0;
                    const int64_t gu = ku >> kOffBits;
                    b = gu < gc || (gu == gc && u < ic);
                }
            }
            better = __builtin_amdgcn_ballot_w64(b) != 0;
        }
        if (!better && lane == 0) {
            const int32_t e = atomicAdd(&list_count[s], 1);
            if (e < list_cap) list[(int64_t)s * list_cap + e] = ic;
            atomicAdd(round_moves, 1);
        }
    }
}

// One wave per taken move.  Grid (kApplyBlocks, S).
__global__ __launch_bounds__(kT) void k_two_opt_apply(
    const int64_t *__restrict__ keys, const int32_t *__restrict__ list, int32_t list_cap,
    const int32_t *__restrict__ list_count, const int32_t *__restrict__ ants, int32_t n, int32_t W,
    int32_t tiles, int32_t round, int32_t *__restrict__ tours, int2 *__restrict__ pxy,
    int64_t *__restrict__ lengths, uint8_t *__restrict__ slots, int32_t *__restrict__ stamp,
    uint32_t *__restrict__ dirty_next, int64_t *__restrict__ gain_sum)
{
    const int32_t s = blockIdx.y;
    const int lane = lane_id();
    const int32_t wave = (int32_t)((blockIdx.x * kT + threadIdx.x) / kWave);
    const int32_t nw = (int32_t)(gridDim.x * (kT / kWave));
    const int32_t cnt = min(list_count[s], list_cap);
    const int32_t ant = ants[s];
    int32_t *tour = tours + (int64_t)ant * n;
    for (int32_t e = wave; e < cnt; e += nw) {
        const int32_t i = list[(int64_t)s * list_cap + e];
        const int64_t key = keys[(int64_t)s * n + i];
        const int32_t o = (int32_t)(key & kOffMask);
        const int64_t g = key >> kOffBits;
        // reverse positions i + 1 .. i + o (each lane swaps its own pairs)
        for (int32_t q = lane; q < o / 2; q += kWave) {
            int32_t p1 = i + 1 + q, p2 = i + o - q;
            p1 -= p1 >= n ? n : 0;
            p2 -= p2 >= n ? n : 0;
            const int32_t v1 = tour[p1], v2 = tour[p2];
            tour[p1] = v2;
            tour[p2] = v1;
            int2 *pc = pxy + (int64_t)s * n;
            const int2 c1 = pc[p1], c2 = pc[p2];
            pc[p1] = c2;
            pc[p2] = c1;
            stamp[(int64_t)s * n + p1] = round;   // the cities at p1 and p2 changed
            stamp[(int64_t)s * n + p2] = round;
        }
        // incoming edges of positions i + 1 .. i + o + 1 changed
        if (slots)
            for (int32_t q = lane; q <= o; q += kWave) {
                int32_t p = i + 1 + q;
                p -= p >= n ? n : 0;
                slots[(int64_t)ant * n + p] = (uint8_t)255;
            }
        // keys of positions i - W .. i + o read a changed position: mark their
        // tiles.  The cyclic range is one or two linear pieces; each covers at
        // most count / kTE + 2 tiles, so 64 lanes suffice (count <= 2W + 1).
        const int32_t first = i - W < 0 ? i - W + n : i - W;
        const int32_t count = W + o + 1;
        const int32_t last = first + count - 1;   // < 2n
        int32_t a1 = first, b1 = last < n ? last : n - 1, b2 = last - n;
        if (count >= n) {
            a1 = 0;
            b1 = n - 1;
            b2 = -1;
        }
        const int32_t t1 = a1 / kTE, nt1 = b1 / kTE - t1 + 1;
        const int32_t nt2 = b2 >= 0 ? b2 / kTE + 1 : 0;
        if (lane < nt1)
            dirty_next[(int64_t)s * tiles + t1 + lane] = 1u;
        else if (lane < nt1 + nt2)
            dirty_next[(int64_t)s * tiles + (lane - nt1)] = 1u;
        if (lane == 0) {
            atomicAdd((unsigned long long *)&lengths[ant], (unsigned long long)g);
            atomicAdd((unsigned long long *)gain_sum, (unsigned long long)g);
        }
    }
}

struct TwoOptLayout {
    int32_t tiles, list_cap;
    size_t sel, ctl, keys, list, dirty, stamp, pxy, total;
    TwoOptLayout(int32_t n, int32_t m, int32_t batch)
    {
        auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
        tiles = (n + kTE - 1) / kTE;   // evaluation tiles (dirty flags)
        list_cap = n / 4 + 1;   // taken spans are disjoint, each >= 4 positions
        sel = 0;
        ctl = up((size_t)m * 4);
        // gain_sum int64, sel_count int32, round_moves int32[16], list_count int32[batch]
        keys = ctl + up(8 + 4 + 4 * kRoundsPerSync + 4 * (size_t)batch);
        list = keys + up((size_t)batch * n * 8);
        dirty = list + up((size_t)batch * list_cap * 4);
        stamp = dirty + up((size_t)2 * batch * tiles * 4);
        pxy = stamp + up((size_t)batch * n * 4);
        total = pxy + up((size_t)batch * n * 8);
    }
};

}  // namespace
}  // namespace aco

using namespace aco;

extern "C" size_t aco_two_opt_workspace_bytes(int32_t n, int32_t m, int32_t batch)
{
    if (n < 1 || m < 1 || batch < 1) return 0;
    return TwoOptLayout(n, m, batch).total;
}

extern "C" int aco_two_opt(const int32_t *xy, int32_t n, int32_t m, int32_t *tours,
                           int64_t *lengths, uint8_t *slots, int32_t window, double p,
                           uint64_t seed, int64_t iteration, int64_t max_rounds, int32_t batch,
                           aco_two_opt_stats_t *stats, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    ACO_REQUIRE(n >= 3 && n <= (1 << 27), "n = %d out of range [3, 2^27]", n);
    ACO_REQUIRE(m >= 1, "m = %d must be >= 1", m);
    ACO_REQUIRE(window >= 1 && window <= ACO_TWO_OPT_MAX_WINDOW, "window = %d out of [1, %d]",
                window, ACO_TWO_OPT_MAX_WINDOW);
    ACO_REQUIRE(std::isfinite(p) && p >= 0.0 && p <= 1.0, "p = %g out of [0, 1]", p);
    ACO_REQUIRE(iteration >= 0 && iteration <= (int64_t)UINT32_MAX, "iteration out of range");
    ACO_REQUIRE(max_rounds >= 0, "max_rounds must be >= 0");
    ACO_REQUIRE(batch >= 1, "batch = %d must be >= 1", batch);
    ACO_REQUIRE(xy && tours && lengths && ws, "NULL array argument");
    const TwoOptLayout lay(n, m, batch);
    if (ws_bytes < lay.total)
        return fail(ACO_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total);
    hipStream_t st = as_stream(stream);
    char *base = (char *)ws;
    int32_t *sel = (int32_t *)(base + lay.sel);
    int64_t *gain_sum = (int64_t *)(base + lay.ctl);
    int32_t *sel_count = (int32_t *)(base + lay.ctl + 8);
    int32_t *round_moves = sel_count + 1;
    int32_t *list_count = round_moves + kRoundsPerSync;
    int64_t *keys = (int64_t *)(base + lay.keys);
    int32_t *list = (int32_t *)(base + lay.list);
    uint32_t *dirty = (uint32_t *)(base + lay.dirty);
    int32_t *stamp = (int32_t *)(base + lay.stamp);
    int2 *pxy = (int2 *)(base + lay.pxy);

    const uint64_t thr = (uint64_t)std::nearbyint(std::ldexp(p, 32));
    k_two_opt_select<<<1, kT, 0, st>>>(seed, (uint32_t)iteration, m, thr, sel, sel_count,
                                       gain_sum);
    ACO_LAUNCH_CHECK("k_two_opt_select");
    int32_t selected = 0;
    ACO_HIP_CHECK(hipMemcpyAsync(&selected, sel_count, 4, hipMemcpyDeviceToHost, st));
    ACO_HIP_CHECK(hipStreamSynchronize(st));

    const int32_t W = window < n / 2 ? window : n / 2;   // each edge pair from its nearer side
    aco_two_opt_stats_t out{selected, 1, 0, 0, 0};
    if (selected > 0 && W >= 2) {
        const size_t np = (size_t)(kTE + W + 2);
        const size_t lds_eval = np * sizeof(int2) + np * 4 +
                                (size_t)(kT / kWave) * (kPosPerWave + W) * 2 + 2 * np;
        const unsigned acc_tiles = blocks_for(n, kT);
        const size_t lds_acc = (size_t)(kT + 2 * W + 2) * sizeof(int64_t);
        for (int32_t c0 = 0; c0 < selected; c0 += batch) {
            const int32_t S = selected - c0 < batch ? selected - c0 : batch;
            const int32_t *ants = sel + c0;
            k_two_opt_init<<<blocks_for((int64_t)S * n, 256), 256, 0, st>>>(
                dirty, lay.tiles, batch, S, stamp, (int64_t)S * n);
            ACO_LAUNCH_CHECK("k_two_opt_init");
            k_two_opt_coords<<<blocks_for((int64_t)S * n, 256), 256, 0, st>>>(xy, tours, ants, n,
                                                                              S, pxy);
            ACO_LAUNCH_CHECK("k_two_opt_coords");
            int64_t r = 0, improving = 0;
            bool done = false, converged = true;
            while (!done) {
                int32_t nb = kRoundsPerSync;
                if (max_rounds > 0 && max_rounds - r + 1 < nb) nb = (int32_t)(max_rounds - r + 1);
                k_two_opt_zero<<<1, 64, 0, st>>>(round_moves, nb);
                ACO_LAUNCH_CHECK("k_two_opt_zero");
                for (int32_t b = 0; b < nb; ++b) {
                    const int64_t rr = r + b;
                    uint32_t *cur = dirty + (size_t)(rr & 1) * batch * lay.tiles;
                    uint32_t *nxt = dirty + (size_t)((rr + 1) & 1) * batch * lay.tiles;
                    k_two_opt_eval<<<dim3(lay.tiles, S), kT, lds_eval, st>>>(
                        pxy, n, W, lay.tiles, (int32_t)rr, stamp, cur, keys, list_count);
                    ACO_LAUNCH_CHECK("k_two_opt_eval");
                    k_two_opt_accept<<<dim3(acc_tiles, S), kT, lds_acc, st>>>(
                        keys, n, W, list, lay.list_cap, list_count, round_moves + b);
                    ACO_LAUNCH_CHECK("k_two_opt_accept");
                    // after max_rounds rounds, one more look only decides convergence
                    if (max_rounds == 0 || rr < max_rounds) {
                        k_two_opt_apply<<<dim3(kApplyBlocks, S), kT, 0, st>>>(
                            keys, list, lay.list_cap, list_count, ants, n, W, lay.tiles,
                            (int32_t)rr, tours, pxy, lengths, slots, stamp, nxt, gain_sum);
                        ACO_LAUNCH_CHECK("k_two_opt_apply");
                    }
                }
                int32_t mv[kRoundsPerSync];
                ACO_HIP_CHECK(
                    hipMemcpyAsync(mv, round_moves, 4 * (size_t)nb, hipMemcpyDeviceToHost, st));
                ACO_HIP_CHECK(hipStreamSynchronize(st));
                for (int32_t b = 0; b < nb && !done; ++b) {
                    if (mv[b] == 0) {
                        done = true;
                    } else if (max_rounds > 0 && r + b == max_rounds) {
                        converged = false;
                        done = true;
                    } else {
                        ++improving;
                        out.moves += mv[b];
                    }
                }
                r += nb;
            }
            out.rounds = improving > out.rounds ? improving : out.rounds;
            out.converged &= converged ? 1 : 0;
        }
        ACO_HIP_CHECK(hipMemcpyAsync(&out.gain, gain_sum, 8, hipMemcpyDeviceToHost, st));
        ACO_HIP_CHECK(hipStreamSynchronize(st));
    }
    if (stats) *stats = out;
    return report_device_error(st);
}
