// Four ants per wave for the batched colonies (k <= 16): the same step as
// build_ant in colony.hpp, with each vector instruction serving four ants.
#pragma once

#include "colony.hpp"

namespace aco {

// ---------------------------------------------------------------------------
// Four ants per wave, for the batched colonies (cities by index, k <= 16, the
// roulette of Eq. 1, full tours).  Ant q runs on lanes [16 q, 16 q + 16), lane
// 16 q + r holding candidate r of that ant's current city.  The FP64 running
// sums are row-local DPP, so one vector instruction serves four ants.  Each
// ant's choice is made exactly as in build_ant (the first slot whose running
// sum passes u S, else the last live slot, else the nearest unvisited city),
// from the same Philox words, so the tours are the same; only the throughput
// differs (a wave's instructions serve four ants where many waves share a SIMD).
// ---------------------------------------------------------------------------
struct Ants4Task {
    const int32_t *xy;     // [n][2]
    const CandW *rows;     // [n][row_stride(k)]
    int32_t n, k;
    uint32_t ant0;         // ant q of the four is ant0 + q * ant_stride
    uint32_t ant_stride;
    int32_t nvalid;        // ants 0 .. nvalid - 1 of the four exist
    uint32_t iteration;
    uint64_t seed;
    int32_t *tours;        // [m][n]
    uint8_t *slots;        // [m][n]
    uint32_t *err;         // the device's error word, or nullptr
};

// LDS of one such wave: four visited bitmasks of set_bytes each (a multiple of
// 16), then the block's Philox words [4][64], staged cities [4][64] and staged
// slots [4][64].
__host__ __device__ __forceinline__ size_t ants4_lds_bytes(size_t set_bytes)
{
    return 4 * set_bytes + 4 * 64 * 4 + 4 * 64 * 4 + 4 * 64;
}

// Lane 15 of each 16-lane row, to every lane of the row (ds_swizzle bit mode
// within 32 lanes: and-mask 0x10, or-mask 0x0F).
__device__ __forceinline__ double row_last_f64(double v)
{
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x1F0);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x1F0);
    return __hiloint2double(hi, lo);
}

template <class GridFn>
__device__ void build_ants4(const Ants4Task &T, unsigned char *lds, size_t set_bytes,
                            const GridFn &grid)
{
    const int lane = lane_id();
    const int q = lane >> 4, gr = lane & 15;
    const int32_t n = T.n, k = T.k;
    const int nv = T.nvalid;
    const int nw = (n + 31) >> 5;                            // words per visited set
    uint32_t *draws = (uint32_t *)(lds + 4 * set_bytes);     // [4][64]
    int32_t *stc = (int32_t *)(draws + 4 * kWave);           // [4][64]
    uint8_t *sts = (uint8_t *)(stc + 4 * kWave);             // [4][64]
    const VisBits vis{(uint32_t *)(lds + (size_t)q * set_bytes)};   // this lane's ant
    const bool mine = q < nv;                                // this lane's ant exists
    const bool active = gr < k && mine;
    const int lr = gr < k ? gr : k - 1;                      // idle lanes re-read a valid element
    const uint64_t row_mask = k >= 16 ? 0xFFFFull : (1ull << k) - 1ull;
    uint64_t act_mask = 0;
    for (int p = 0; p < nv; ++p) act_mask |= row_mask << (16 * p);
    const GridView g = grid();

    for (int p = 0; p < 4; ++p) {
        uint32_t *w = (uint32_t *)(lds + (size_t)p * set_bytes);
        for (int i = lane; i < nw; i += kWave) w[i] = 0u;
    }
    // the block's words: draws[p][l] is ant p's word for step base + l
    auto fill_draws = [&](int32_t base) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
            draws[p * kWave + lane] = colony_draw(T.seed, T.iteration,
                                                  T.ant0 + (uint32_t)p * T.ant_stride,
                                                  (uint32_t)(base + lane));
    };
    fill_draws(0);
    int32_t c = (int32_t)(((uint64_t)draws[q * kWave] * (uint64_t)n) >> 32);   // start city
    const int32_t start = c;
    if (gr == 0 && mine) vis.set(c);

    constexpr int32_t ks = row_stride(16);   // k <= 16
    CandW eg = T.rows[(int64_t)c * ks + lr], en = eg;
    bool hit = true;
    for (int32_t base = 0; base < n; base += kWave) {
        if (base > 0) fill_draws(base);
        const int32_t last = min(base + kWave - 1, n - 1);
        if (base == 0 && gr == 0) {   // step 0: the start city, no construction record
            stc[q * kWave] = start;
            sts[q * kWave] = (uint8_t)kNoSlot;
        }
        for (int32_t step = max(base, 1); step <= last; ++step) {
            const int idx = step - base;
            const CandW e = hit ? eg : en;
            const int32_t j = e.city;
            const uint32_t seen = vis.test(j);
            const uint32_t xw = draws[q * kWave + idx];
            const bool live = active && seen == 0u && e.w > 0.0f;
            const uint64_t any = __builtin_amdgcn_ballot_w64(seen == 0u) &
                                 __builtin_amdgcn_ballot_w64(e.w > 0.0f) & act_mask;
            // this lane's ant's live slots (each lane reads its own row's bits)
            const uint32_t aq = (uint32_t)(any >> (16 * q)) & 0xFFFFu;
            // each ant's first live candidate (or its row's lane 15) is guessed;
            // the four rows go out in one load while the scan runs
            const int32_t guess = __shfl(j, (lane & 48) + __builtin_ctz(aq | 0x8000u));
            eg = T.rows[(int64_t)guess * ks + lr];
            const double wv = live ? (double)e.w : 0.0;
            const double u = (double)xw * 0x1p-32;
            const double cum = wave_incl_scan_f64(wv, 16);
            // S: lane 15's running sum equals lane k - 1's (later lanes add zeros)
            const double S = row_last_f64(cum);
            const uint64_t pass = __builtin_amdgcn_ballot_w64(u * S < cum) & any;
            // each ant's slot: the first whose running sum passes u S, else the
            // last live one
            const uint32_t hq = (uint32_t)(pass >> (16 * q)) & 0xFFFFu;
            const int f = hq ? __builtin_ctz(hq) : 31 - __builtin_clz(aq | 1u);
            int32_t jn = __shfl(j, (lane & 48) + f);
            uint32_t sl = aq ? (uint32_t)f : kNoSlot;
            // ants with no live candidate: the nearest unvisited city, one at a time
            const uint64_t fbm = __builtin_amdgcn_ballot_w64(aq == 0u && mine);
            uint32_t need_fb = (uint32_t)(fbm & 1u) | (uint32_t)((fbm >> 15) & 2u) |
                               (uint32_t)((fbm >> 30) & 4u) | (uint32_t)((fbm >> 45) & 8u);
            while (need_fb) {
                const int p = __builtin_ctz(need_fb);
                need_fb &= need_fb - 1u;
                const VisBits vp{(uint32_t *)(lds + (size_t)p * set_bytes)};
                const int32_t jp = fallback_city(g, T.xy, read_lane_i32(c, 16 * p),
                                                 [&](int city) { return vp.test(city); });
                jn = q == p ? jp : jn;
            }
            // always in range; the guard keeps a logic error in bounds and
            // reports it (a branch that is never taken: no register held
            // across the loop, which would cost spills at this occupancy)
            const bool out = (uint32_t)jn >= (uint32_t)n;
            if (__builtin_expect(out && mine, 0)) flag_error(T.err, kErrNextCity);
            jn = out ? start : jn;
            hit = jn == guess;
            if (!hit) en = T.rows[(int64_t)jn * ks + lr];
            if (gr == 0 && mine) {
                vis.set(jn);
                stc[q * kWave + idx] = jn;
                sts[q * kWave + idx] = (uint8_t)sl;
            }
            c = jn;
        }
        // the block's records out, ant by ant
        for (int p = 0; p < nv; ++p) {
            if (base + lane <= last) {
                const int64_t a = (int64_t)T.ant0 + (int64_t)p * T.ant_stride;
                T.tours[a * n + base + lane] = stc[p * kWave + lane];
                T.slots[a * n + base + lane] = sts[p * kWave + lane];
            }
        }
    }
}

}  // namespace aco
