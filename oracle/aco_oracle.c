/*
 * CPU oracle for the ACO hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct reference of what the GPU path computes:
 * Ant System tour construction with the random proportional rule (Eq. 1),
 * evaporation (Eq. 2) and the all-ant 1/L deposit (Eq. 3-4), with pheromone
 * stored only on each city's k nearest-neighbour candidate edges.
 * Floating point is FP64 except where the method fixes FP32 (the stored
 * pheromone and its update).  The fallback when every candidate is visited is
 * an O(n) brute-force scan.  Nothing here is shared with the GPU library, and
 * only the test suite, the smoke check and the benchmark's CPU baseline may
 * load it.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Distances (Section 2: complete graph with symmetric d_ij = d_ji).    */
/* d_ij = nint(sqrt((xi-xj)^2 + (yi-yj)^2)), an integer.                */
/* ------------------------------------------------------------------ */

int64_t oracle_sq(const int32_t *xy, int64_t i, int64_t j)
{
    int64_t dx = (int64_t)xy[2 * i] - (int64_t)xy[2 * j];
    int64_t dy = (int64_t)xy[2 * i + 1] - (int64_t)xy[2 * j + 1];
    return dx * dx + dy * dy;
}

/* floor(sqrt(s)) exactly, for 0 <= s < 2^63. */
static uint64_t isqrt_floor(uint64_t s)
{
    uint64_t r = (uint64_t)sqrt((double)s);
    while (r * r > s) r--;
    while ((r + 1) * (r + 1) <= s) r++;
    return r;
}

/* nint(sqrt(s)): sqrt(s) >= r + 1/2  <=>  s > r^2 + r for integer s, r = floor(sqrt(s)).
 * (sqrt(s) is never exactly r + 1/2 for integer s.) */
int64_t oracle_nint_sqrt(int64_t s)
{
    uint64_t r = isqrt_floor((uint64_t)s);
    return (int64_t)((uint64_t)s - r * r > r ? r + 1 : r);
}

int64_t oracle_dist(const int32_t *xy, int64_t i, int64_t j)
{
    return oracle_nint_sqrt(oracle_sq(xy, i, j));
}

int64_t oracle_tour_length(const int32_t *xy, int64_t n, const int32_t *tour)
{
    int64_t L = 0;
    for (int64_t t = 0; t < n; t++) L += oracle_dist(xy, tour[t], tour[(t + 1) % n]);
    return L;
}

/* ------------------------------------------------------------------ */
/* Candidate lists (Section 6, the candidate-list idea of ACS: only the  */
/* closest cities are considered).  nn[i] = the k smallest keys          */
/* (d_ij, j) over j != i, ascending by distance then index.             */
/* ------------------------------------------------------------------ */

static int key_less(int64_t d1, int64_t j1, int64_t d2, int64_t j2)
{
    return d1 < d2 || (d1 == d2 && j1 < j2);
}

static void knn_row(const int32_t *xy, int64_t n, int k, int64_t i, int32_t *nn, int32_t *nnd)
{
    int cnt = 0;
    for (int64_t j = 0; j < n; j++) {
        if (j == i) continue;
        int64_t d = oracle_dist(xy, i, j);
        if (cnt == k && !key_less(d, j, nnd[k - 1], nn[k - 1])) continue;
        int p = cnt < k ? cnt++ : k - 1;          /* insertion sort into the first k */
        while (p > 0 && key_less(d, j, nnd[p - 1], nn[p - 1])) {
            nn[p] = nn[p - 1];
            nnd[p] = nnd[p - 1];
            p--;
        }
        nn[p] = (int32_t)j;
        nnd[p] = (int32_t)d;
    }
}

/* Rows `rows[0..count)` of the candidate table; out arrays are [count][k]. */
void oracle_knn_rows(const int32_t *xy, int64_t n, int k, const int32_t *rows, int64_t count,
                     int32_t *nn, int32_t *nnd)
{
    for (int64_t q = 0; q < count; q++)
        knn_row(xy, n, k, rows[q], nn + q * k, nnd + q * k);
}

typedef struct {
    const int32_t *xy;
    int64_t n;
    int k;
    const int32_t *rows;
    int64_t lo, hi;
    int32_t *nn, *nnd;
} knn_job_t;

static void *knn_worker(void *arg)
{
    knn_job_t *J = (knn_job_t *)arg;
    for (int64_t q = J->lo; q < J->hi; q++)
        knn_row(J->xy, J->n, J->k, J->rows[q], J->nn + q * J->k, J->nnd + q * J->k);
    return NULL;
}

/* The same rows split over `threads` threads (contiguous blocks of rows). */
void oracle_knn_rows_mt(const int32_t *xy, int64_t n, int k, const int32_t *rows, int64_t count,
                        int32_t *nn, int32_t *nnd, int threads)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    knn_job_t jobs[256];
    for (int t = 0; t < threads; t++) {
        jobs[t] = (knn_job_t){xy, n, k, rows, count * t / threads, count * (t + 1) / threads,
                              nn, nnd};
        pthread_create(&th[t], NULL, knn_worker, &jobs[t]);
    }
    for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
}

/* rev[i][r] = position of i in nn[nn[i][r]], or -1 when i is not a candidate of nn[i][r]. */
void oracle_rev(int64_t n, int k, const int32_t *nn, int8_t *rev)
{
    for (int64_t i = 0; i < n; i++)
        for (int r = 0; r < k; r++) {
            int64_t j = nn[i * k + r];
            rev[i * k + r] = -1;
            for (int s = 0; s < k; s++)
                if (nn[j * k + s] == i) { rev[i * k + r] = (int8_t)s; break; }
        }
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the   */
/* Philox S-box on a 4x32-bit counter with a 2x32-bit key bumped by the  */
/* Weyl constants between rounds.                                        */
/* ------------------------------------------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The colony's random word for (seed, iteration, ant, step):
 * counter = (step, ant, iteration, 0), key = (seed low, seed high), word 0. */
uint32_t oracle_draw(uint64_t seed, int64_t iteration, int64_t ant, int64_t step)
{
    uint32_t ctr[4] = {(uint32_t)step, (uint32_t)ant, (uint32_t)iteration, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[0];
}

/* Random start city (Section 2: ants start at a random city): (x * n) >> 32. */
int64_t oracle_start_city(uint64_t seed, int64_t iteration, int64_t ant, int64_t n)
{
    return (int64_t)(((uint64_t)oracle_draw(seed, iteration, ant, 0) * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------ */
/* Fallback when every candidate of c is visited: the nearest unvisited */
/* city, key (d_cj, j).  Brute force over all n cities.  Two passes:    */
/* the smallest squared distance s_min fixes d* = nint(sqrt(s_min)); a  */
/* city has d <= d* exactly when s <= d*^2 + d*, and the lowest index    */
/* among those is the minimum key.                                      */
/* ------------------------------------------------------------------ */

static int64_t nearest_unvisited(const int32_t *xy, int64_t n, int64_t c, const uint8_t *vis,
                                 int64_t *d_out)
{
    int64_t smin = -1;
    for (int64_t j = 0; j < n; j++) {
        if (vis[j]) continue;
        int64_t s = oracle_sq(xy, c, j);
        if (smin < 0 || s < smin) smin = s;
    }
    if (smin < 0) return -1;
    int64_t dstar = oracle_nint_sqrt(smin);
    int64_t thresh = dstar * dstar + dstar;
    for (int64_t j = 0; j < n; j++)
        if (!vis[j] && oracle_sq(xy, c, j) <= thresh) { *d_out = dstar; return j; }
    return -1; /* unreachable */
}

/* Plain definition, for pinning the two-pass scan: argmin of (nint d, j). */
int64_t oracle_nearest_unvisited_plain(const int32_t *xy, int64_t n, int64_t c, const uint8_t *vis)
{
    int64_t best = -1, bd = 0;
    for (int64_t j = 0; j < n; j++) {
        if (vis[j]) continue;
        int64_t d = oracle_dist(xy, c, j);
        if (best < 0 || d < bd) { best = j; bd = d; }
    }
    return best;
}

int64_t oracle_nearest_unvisited(const int32_t *xy, int64_t n, int64_t c, const uint8_t *vis)
{
    int64_t d;
    return nearest_unvisited(xy, n, c, vis, &d);
}

/* The same minimum key, found by a sweep outward from c along the cities in
 * order of x: a shortcut for checking long tours, pinned against the brute
 * force above.  xorder lists every city by ascending x (any order among
 * equal x) and xpos[c] is c's place in that list.  A city with
 * |x_j - x_c| > D (integers) has sqrt(s) >= D + 1 and so d_cj > D: once the
 * nearer of the two next cities is further than the best distance found in
 * x alone, no remaining city can have a smaller or equal distance. */
static int64_t nearest_unvisited_sweep(const int32_t *xy, int64_t n, int64_t c,
                                       const uint8_t *vis, const int32_t *xorder,
                                       const int32_t *xpos, int64_t *d_out)
{
    int64_t best = -1, bd = 0;
    int64_t lo = (int64_t)xpos[c] - 1, hi = (int64_t)xpos[c] + 1;
    int64_t xc = xy[2 * c];
    for (;;) {
        int64_t dl = lo >= 0 ? xc - xy[2 * (int64_t)xorder[lo]] : -1;   /* >= 0 when present */
        int64_t dh = hi < n ? xy[2 * (int64_t)xorder[hi]] - xc : -1;
        if (dl < 0 && dh < 0) break;
        int use_lo = dh < 0 || (dl >= 0 && dl <= dh);
        int64_t dx = use_lo ? dl : dh;
        if (best >= 0 && dx > bd) break;
        int64_t j = xorder[use_lo ? lo-- : hi++];
        if (vis[j]) continue;
        int64_t d = oracle_dist(xy, c, j);
        if (best < 0 || d < bd || (d == bd && j < best)) { best = j; bd = d; }
    }
    *d_out = bd;
    return best;
}

int64_t oracle_nearest_unvisited_sweep(const int32_t *xy, int64_t n, int64_t c,
                                       const uint8_t *vis, const int32_t *xorder,
                                       const int32_t *xpos)
{
    int64_t d;
    return nearest_unvisited_sweep(xy, n, c, vis, xorder, xpos, &d);
}

/* ------------------------------------------------------------------ */
/* Nearest-neighbour tour from city 0 (pheromone initialisation).       */
/* Each step takes the unvisited city with the smallest (d, j).  Every  */
/* candidate key is smaller than every non-candidate key, so the first  */
/* unvisited entry of nn[c] is that city whenever one exists.           */
/* ------------------------------------------------------------------ */

int64_t oracle_nn_tour(const int32_t *xy, int64_t n, int k, const int32_t *nn, const int32_t *nnd,
                       int32_t *tour)
{
    uint8_t *vis = (uint8_t *)calloc((size_t)n, 1);
    int64_t c = 0, L = 0;
    vis[0] = 1;
    tour[0] = 0;
    for (int64_t t = 1; t < n; t++) {
        int64_t j = -1, d = 0;
        for (int r = 0; r < k; r++)
            if (!vis[nn[c * k + r]]) { j = nn[c * k + r]; d = nnd[c * k + r]; break; }
        if (j < 0) j = nearest_unvisited(xy, n, c, vis, &d);
        vis[j] = 1;
        tour[t] = (int32_t)j;
        L += d;
        c = j;
    }
    L += oracle_dist(xy, c, 0);
    free(vis);
    return L;
}

/* The plain definition: argmin over all unvisited cities at every step (O(n^2)). */
int64_t oracle_nn_tour_plain(const int32_t *xy, int64_t n, int32_t *tour)
{
    uint8_t *vis = (uint8_t *)calloc((size_t)n, 1);
    int64_t c = 0;
    vis[0] = 1;
    tour[0] = 0;
    for (int64_t t = 1; t < n; t++) {
        int64_t j = oracle_nearest_unvisited_plain(xy, n, c, vis);
        vis[j] = 1;
        tour[t] = (int32_t)j;
        c = j;
    }
    free(vis);
    return oracle_tour_length(xy, n, tour);
}

/* Initial pheromone: tau0 = 1 / (n * L_nn), rounded once to FP32. */
float oracle_tau0(int64_t n, int64_t L_nn)
{
    return (float)(1.0 / ((double)n * (double)L_nn));
}

/* ------------------------------------------------------------------ */
/* Tour construction, Eq. 1 (random proportional rule).                 */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    int k;
    const int32_t *xy;
    const int32_t *nn;
    const int32_t *nnd;
    const float *tau;        /* [n][k] FP32 pheromone */
    const double *eta;       /* [n][k] heuristic override, or NULL for eta = 1/max(d,1) */
    double alpha, beta;
    uint64_t seed;
    int64_t iteration;
    int sampler;             /* 0: roulette of Eq. 1; 1: Independent Roulette (Section 3) */
    const int32_t *xorder;   /* replay only: cities by x for the sweep check, or NULL */
    const int32_t *xpos;
} colony_t;

/* Heuristic eta_ir = 1/d_ir (Section 2); d = 0 (coincident cities) is read as 1. */
static double eta_of(const colony_t *C, int64_t c, int r)
{
    if (C->eta) return C->eta[c * C->k + r];
    int64_t d = C->nnd[c * C->k + r];
    return 1.0 / (double)(d > 1 ? d : 1);
}

/* Weight tau^alpha * eta^beta of candidate r of city c, in FP64. */
static double weight_of(const colony_t *C, int64_t c, int r)
{
    return pow((double)C->tau[c * C->k + r], C->alpha) * pow(eta_of(C, c, r), C->beta);
}

/* The roulette over the unvisited candidates of c.
 * w[r] is the weight (0 for visited slots), cum[r] the running sum over
 * unvisited slots in rank order.  Returns S = the total. */
static double row_weights(const colony_t *C, int64_t c, const uint8_t *vis, double *w, double *cum,
                          int *n_unvisited)
{
    double S = 0.0;
    int nu = 0;
    for (int r = 0; r < C->k; r++) {
        int64_t j = C->nn[c * C->k + r];
        w[r] = 0.0;
        if (!vis[j]) { w[r] = weight_of(C, c, r); nu++; }
        S += w[r];
        cum[r] = S;
    }
    *n_unvisited = nu;
    return S;
}

/* Pick the first unvisited slot with u*S < cum[r]; if rounding leaves none,
 * the last slot with positive weight.  A zero-weight slot is never chosen. */
static int roulette(const colony_t *C, const double *w, const double *cum, double S, double u)
{
    double target = u * S;
    int last = -1;
    for (int r = 0; r < C->k; r++) {
        if (w[r] <= 0.0) continue;
        if (target < cum[r]) return r;
        last = r;
    }
    return last;
}

/* Independent Roulette (Section 3): every unvisited candidate r with w_r > 0
 * gets its own uniform U_r and the largest w_r * U_r (FP64) wins, ties to
 * the lower rank.  U_r = x * 2^-32, x = word (r mod 4) of the Philox block at
 * counter (t, ant, iteration, 1 + r / 4) (word 3 of the roulette's counter is
 * 0, so the two never share a draw).  *v_best and *v_second receive the two
 * largest products. */
static double ir_uniform(const colony_t *C, int64_t ant, int64_t t, int r)
{
    uint32_t ctr[4] = {(uint32_t)t, (uint32_t)ant, (uint32_t)C->iteration, 1u + (uint32_t)(r / 4)};
    uint32_t key[2] = {(uint32_t)C->seed, (uint32_t)(C->seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return (double)out[r % 4] * 0x1p-32;
}

static int independent_roulette(const colony_t *C, int64_t ant, int64_t t, const double *w,
                                double *v_best, double *v_second, double *v_of)
{
    int best = -1;
    double vb = -1.0, vs = -1.0;
    for (int r = 0; r < C->k; r++) {
        v_of[r] = -1.0;
        if (w[r] <= 0.0) continue;
        double v = w[r] * ir_uniform(C, ant, t, r);
        v_of[r] = v;
        if (v > vb) { vs = vb; vb = v; best = r; }
        else if (v > vs) vs = v;
    }
    *v_best = vb;
    *v_second = vs;
    return best;
}

/* The slot chosen at tour position t with draw u (roulette) or the step's
 * independent uniforms (Independent Roulette). */
static int select_slot(const colony_t *C, int64_t ant, int64_t t, const double *w,
                       const double *cum, double S, double u)
{
    if (C->sampler == 0) return roulette(C, w, cum, S, u);
    double vb, vs, v_of[64];
    return independent_roulette(C, ant, t, w, &vb, &vs, v_of);
}

typedef struct {
    int64_t length;
    int64_t fallbacks;
} ant_result_t;

/* Build one ant's tour.  slot[t] = rank of tour[t] in nn[tour[t-1]] or -1 for a
 * fallback move (slot[0] = -1); prob[t] = probability of the move (-1 for a fallback). */
static ant_result_t construct_ant(const colony_t *C, int64_t ant, int32_t *tour, int8_t *slot,
                                  double *prob)
{
    int64_t n = C->n;
    int k = C->k;
    uint8_t *vis = (uint8_t *)calloc((size_t)n, 1);
    double w[64], cum[64];
    ant_result_t res = {0, 0};
    int64_t c = oracle_start_city(C->seed, C->iteration, ant, n);
    int64_t start = c;
    vis[c] = 1;
    tour[0] = (int32_t)c;
    if (slot) slot[0] = -1;
    if (prob) prob[0] = 1.0;
    for (int64_t t = 1; t < n; t++) {
        double u = (double)oracle_draw(C->seed, C->iteration, ant, t) * 0x1p-32;
        int nu;
        double S = row_weights(C, c, vis, w, cum, &nu);
        int64_t j, d;
        if (nu > 0 && S > 0.0) {
            int r = select_slot(C, ant, t, w, cum, S, u);
            j = C->nn[c * k + r];
            d = C->nnd[c * k + r];
            if (slot) slot[t] = (int8_t)r;
            if (prob) prob[t] = w[r] / S;
        } else {
            j = nearest_unvisited(C->xy, n, c, vis, &d);
            res.fallbacks++;
            if (slot) slot[t] = -1;
            if (prob) prob[t] = -1.0;
        }
        vis[j] = 1;
        tour[t] = (int32_t)j;
        res.length += d;
        c = j;
    }
    res.length += oracle_dist(C->xy, c, start);
    free(vis);
    return res;
}

/* Teacher-forced replay of a given tour.  At every step the oracle computes its
 * own probabilities and choice, compares with the move the tour takes, and then
 * follows the given tour.  Counters (out[0..7]):
 *   0 steps checked, 1 fallback steps, 2 choice mismatches at a near boundary
 *   (|u - C_r/S| < boundary_eps for some unvisited r), 3 hard mismatches,
 *   4 fallback mismatches, 5 invalid moves (revisit / out of range / wrong start),
 *   6 steps where u is within boundary_eps of a cumulative boundary (any outcome).
 * prob[t] receives the oracle's probability of the move the tour takes
 * (-1 for a fallback step, 0 if the move has zero probability). */
/* Replay of steps first..n-1 of `tour` after its first `first` cities have
 * been marked visited (they are checked by the caller). */
static void replay_from(const colony_t *C, int64_t ant, const int32_t *tour, int64_t first,
                        double boundary_eps, double *prob, int64_t *out)
{
    int64_t n = C->n;
    int k = C->k;
    uint8_t *vis = (uint8_t *)calloc((size_t)n, 1);
    double w[64], cum[64];
    int64_t c = -1;
    for (int64_t t = 0; t < first; t++) {
        c = tour[t];
        if (c < 0 || c >= n || vis[c]) { out[5]++; free(vis); return; }
        vis[c] = 1;
        prob[t] = 1.0;
    }
    for (int64_t t = first; t < n; t++) {
        int64_t j = tour[t];
        out[0]++;
        if (j < 0 || j >= n || vis[j]) { out[5]++; prob[t] = 0.0; break; }
        double u = (double)oracle_draw(C->seed, C->iteration, ant, t) * 0x1p-32;
        int nu;
        double S = row_weights(C, c, vis, w, cum, &nu);
        if (nu > 0 && S > 0.0) {
            int taken = -1;
            for (int q = 0; q < k; q++)
                if (C->nn[c * k + q] == j) taken = q;
            prob[t] = (taken >= 0) ? w[taken] / S : 0.0;
            int r, near = 0;
            if (C->sampler == 0) {
                r = roulette(C, w, cum, S, u);
                for (int q = 0; q < k; q++)
                    if (w[q] > 0.0 && fabs(u - cum[q] / S) < boundary_eps) near = 1;
            } else {
                /* a near tie: the top two products within 2^-22 of each other
                 * (the GPU's weights are the FP64 weights rounded once to FP32) */
                double vb, vs, v_of[64];
                r = independent_roulette(C, ant, t, w, &vb, &vs, v_of);
                if (vs >= 0.0 && vb - vs <= 0x1p-22 * vb) near = 1;
                if (taken >= 0 && taken != r && v_of[taken] >= 0.0 &&
                    vb - v_of[taken] > 0x1p-22 * vb) near = 0;
                prob[t] = (taken >= 0 && v_of[taken] >= 0.0) ? v_of[taken] / vb : 0.0;
            }
            if (near) out[6]++;
            if (taken != r) {
                if (near && taken >= 0 && w[taken] > 0.0) out[2]++;
                else out[3]++;
            }
        } else {
            int64_t d, want;
            out[1]++;
            prob[t] = -1.0;
            if (C->xorder)
                want = nearest_unvisited_sweep(C->xy, n, c, vis, C->xorder, C->xpos, &d);
            else
                want = nearest_unvisited(C->xy, n, c, vis, &d);
            if (want != j) out[4]++;
        }
        vis[j] = 1;
        c = j;
    }
    free(vis);
}

void oracle_replay_ant(const colony_t *C, int64_t ant, const int32_t *tour, double boundary_eps,
                       double *prob, int64_t *out)
{
    memset(out, 0, 8 * sizeof(int64_t));
    if (tour[0] != oracle_start_city(C->seed, C->iteration, ant, C->n)) out[5]++;
    replay_from(C, ant, tour, 1, boundary_eps, prob, out);
}

/* ------------------------------------------------------------------ */
/* Pheromone from the ants' local best tours (the P-ACO variant of        */
/* Section 3): no evaporation; an edge of ant a's local best contributes  */
/* the quality ratio w_a = L_g / L_a in (0, 1], L_g the shortest local    */
/* best, so tau = tau_base + delta * sum of w_a over the local bests that */
/* use the edge.  w_a is quantised as q_a = floor(2^shift * w_a) with the */
/* ratio in FP64; tau = fl32(base + fl32(fl32(acc) * fl32(delta 2^-shift))).*/
/* ------------------------------------------------------------------ */

static void deposit_quanta(int64_t n, int k, const int32_t *nn, int64_t m, const int32_t *tours,
                           const int64_t *qa, int64_t *acc);

void oracle_pheromone_local_best(int64_t n, int k, const int32_t *nn, int64_t m,
                                 const int32_t *lbest, const int64_t *lbest_len, double tau_base,
                                 double delta, int shift, float *tau, int64_t *q_out)
{
    int64_t Lg = lbest_len[0];
    for (int64_t a = 1; a < m; a++)
        if (lbest_len[a] < Lg) Lg = lbest_len[a];
    int64_t *q = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    for (int64_t a = 0; a < m; a++) {
        double ratio = (double)Lg / (double)lbest_len[a];
        q[a] = (int64_t)floor(ldexp(ratio, shift));
        if (q_out) q_out[a] = q[a];
    }
    int64_t *acc = (int64_t *)malloc((size_t)(n * k) * sizeof(int64_t));
    deposit_quanta(n, k, nn, m, lbest, q, acc);
    float base = (float)tau_base;
    float scale = (float)(delta * ldexp(1.0, -shift));
    for (int64_t e = 0; e < n * k; e++) {
        float dep = (float)acc[e] * scale;
        tau[e] = base + dep;
    }
    free(acc);
    free(q);
}

/* ------------------------------------------------------------------ */
/* PartialACO (Section 3.1, Algorithm 1): each ant keeps a random part   */
/* of its local best tour and rebuilds the rest.  The plan of ant a at   */
/* an iteration comes from the Philox block at counter (0, a, iteration):*/
/*   word 0: start position s = (x0 n) >> 32 in the local best tour (for */
/*           a full construction this is the usual start city);          */
/*   word 1: the ant only partially modifies its tour when x1 < P, with  */
/*           P = round(p 2^32) for the probability p (Section 4);        */
/*   word 2: it rebuilds r = 1 + ((x2 M) >> 32) cities, uniform in       */
/*           [1, M], M the cap on the modified share (Section 4).         */
/* The kept part is lbest[s], ..., lbest[s + n - r - 1] (cyclic); the   */
/* rest is constructed with Eq. 1 from the last kept city, the step at  */
/* tour position t drawing from counter (t, a, iteration) as always.     */
/* ------------------------------------------------------------------ */

void oracle_partial_plan(uint64_t seed, int64_t iteration, int64_t ant, int64_t n,
                         uint64_t p_threshold, int64_t max_modify, int64_t *start,
                         int *partial, int64_t *rebuild)
{
    uint32_t ctr[4] = {0u, (uint32_t)ant, (uint32_t)iteration, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    int64_t M = max_modify < 1 ? 1 : (max_modify > n - 1 ? n - 1 : max_modify);
    *start = (int64_t)(((uint64_t)w[0] * (uint64_t)n) >> 32);
    *partial = (uint64_t)w[1] < p_threshold;
    *rebuild = 1 + (int64_t)(((uint64_t)w[2] * (uint64_t)M) >> 32);
}

static ant_result_t construct_partial_ant(const colony_t *C, int64_t ant, const int32_t *lbest,
                                          uint64_t p_threshold, int64_t max_modify,
                                          int32_t *tour, int8_t *slot, double *prob)
{
    int64_t n = C->n, s, r;
    int partial;
    oracle_partial_plan(C->seed, C->iteration, ant, n, p_threshold, max_modify, &s, &partial, &r);
    if (!partial) return construct_ant(C, ant, tour, slot, prob);
    int k = C->k;
    int64_t keep = n - r;
    uint8_t *vis = (uint8_t *)calloc((size_t)n, 1);
    double w[64], cum[64];
    ant_result_t res = {0, 0};
    int64_t c = -1;
    for (int64_t t = 0; t < keep; t++) {
        c = lbest[(s + t) % n];
        vis[c] = 1;
        tour[t] = (int32_t)c;
        if (slot) slot[t] = -1;
        if (prob) prob[t] = 1.0;
        if (t > 0) res.length += oracle_dist(C->xy, tour[t - 1], c);
    }
    for (int64_t t = keep; t < n; t++) {
        double u = (double)oracle_draw(C->seed, C->iteration, ant, t) * 0x1p-32;
        int nu;
        double S = row_weights(C, c, vis, w, cum, &nu);
        int64_t j, d;
        if (nu > 0 && S > 0.0) {
            int q = select_slot(C, ant, t, w, cum, S, u);
            j = C->nn[c * k + q];
            d = C->nnd[c * k + q];
            if (slot) slot[t] = (int8_t)q;
            if (prob) prob[t] = w[q] / S;
        } else {
            j = nearest_unvisited(C->xy, n, c, vis, &d);
            res.fallbacks++;
            if (slot) slot[t] = -1;
            if (prob) prob[t] = -1.0;
        }
        vis[j] = 1;
        tour[t] = (int32_t)j;
        res.length += d;
        c = j;
    }
    res.length += oracle_dist(C->xy, c, tour[0]);
    free(vis);
    return res;
}

void oracle_construct_partial(int64_t n, int k, const int32_t *xy, const int32_t *nn,
                              const int32_t *nnd, const float *tau, const double *eta,
                              double alpha, double beta, uint64_t seed, int64_t iteration,
                              const int64_t *ants, int64_t count, const int32_t *lbest,
                              uint64_t p_threshold, int64_t max_modify, int sampler,
                              int32_t *tours, int64_t *lengths, int8_t *slots, double *probs)
{
    colony_t C;
    C.n = n; C.k = k; C.xy = xy; C.nn = nn; C.nnd = nnd; C.tau = tau; C.eta = eta;
    C.alpha = alpha; C.beta = beta; C.seed = seed; C.iteration = iteration;
    C.sampler = sampler;
    C.xorder = NULL;
    C.xpos = NULL;
    for (int64_t q = 0; q < count; q++) {
        ant_result_t r = construct_partial_ant(&C, ants[q], lbest + q * n, p_threshold,
                                               max_modify, tours + q * n,
                                               slots ? slots + q * n : NULL,
                                               probs ? probs + q * n : NULL);
        lengths[q] = r.length;
    }
}

/* Teacher-forced replay of a PartialACO tour: the kept part must be the
 * planned segment of lbest (each wrong city counts as invalid, out[5]);
 * the rebuilt steps are replayed as in oracle_replay_ant.  out[7] receives
 * the number of kept cities (n for none when the ant built a full tour:
 * then the whole tour is replayed from its start city). */
void oracle_replay_partial(int64_t n, int k, const int32_t *xy, const int32_t *nn,
                           const int32_t *nnd, const float *tau, const double *eta, double alpha,
                           double beta, uint64_t seed, int64_t iteration, int64_t ant,
                           const int32_t *lbest, uint64_t p_threshold, int64_t max_modify,
                           int sampler, const int32_t *tour, double boundary_eps, double *prob,
                           int64_t *out)
{
    colony_t C;
    C.n = n; C.k = k; C.xy = xy; C.nn = nn; C.nnd = nnd; C.tau = tau; C.eta = eta;
    C.alpha = alpha; C.beta = beta; C.seed = seed; C.iteration = iteration;
    C.sampler = sampler;
    C.xorder = NULL;
    C.xpos = NULL;
    int64_t s, r;
    int partial;
    oracle_partial_plan(seed, iteration, ant, n, p_threshold, max_modify, &s, &partial, &r);
    if (!partial) {
        oracle_replay_ant(&C, ant, tour, boundary_eps, prob, out);
        out[7] = n;
        return;
    }
    memset(out, 0, 8 * sizeof(int64_t));
    int64_t keep = n - r;
    for (int64_t t = 0; t < keep; t++)
        if (tour[t] != lbest[(s + t) % n]) out[5]++;
    replay_from(&C, ant, tour, keep, boundary_eps, prob, out);
    out[7] = keep;
}

/* ------------------------------------------------------------------ */
/* Windowed 2-opt local search.  Section 4 applies 2-opt to a tour with */
/* a small probability (0.001); Section 5 restricts it to pairs of tour */
/* edges at most W = 500 positions apart.  The paper fixes neither the  */
/* move order nor how the chosen tours are drawn; this is the reading:  */
/*                                                                      */
/* A tour takes part when word 3 of the Philox block at counter         */
/* (0, ant, iteration, 0) is below P = round(p 2^32) (words 0-2 are the */
/* start city and PartialACO's plan).                                   */
/*                                                                      */
/* Move (i, o), 2 <= o <= W' = min(W, n/2), positions mod n, j = i + o: */
/* drop the edges (t_i, t_i+1) and (t_j, t_j+1), add (t_i, t_j) and     */
/* (t_i+1, t_j+1), i.e. reverse t_i+1 .. t_j.  Its gain is              */
/*   g = d(t_i, t_j) + d(t_i+1, t_j+1) - d(t_i, t_i+1) - d(t_j, t_j+1), */
/* the change of the tour length.  It touches positions i .. j+1, its   */
/* span.  One round: every position i takes its best move (the smallest */
/* g < 0, ties to the smaller o); a position's move is applied when no  */
/* other position's move with an overlapping span is better by (g, i).  */
/* Applied spans are disjoint, so the moves commute and their gains     */
/* add.  Rounds repeat until no position has a move with g < 0: the     */
/* tour is then 2-optimal for every pair of edges within W positions.   */
/* ------------------------------------------------------------------ */

int oracle_two_opt_selected(uint64_t seed, int64_t iteration, int64_t ant, uint64_t p_threshold)
{
    uint32_t ctr[4] = {0u, (uint32_t)ant, (uint32_t)iteration, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    return (uint64_t)w[3] < p_threshold;
}

/* W' = min(W, floor(n/2)): a pair of edges o positions apart one way is   */
/* n - o apart the other way, so it is taken once, from the nearer side    */
/* (twice when o = n/2); o = n - 1 would pair adjacent edges.              */
static int64_t two_opt_window(int64_t n, int64_t window)
{
    return window < n / 2 ? window : n / 2;
}

/* gain of move (i, o) on the tour, straight from the definition */
static int64_t two_opt_gain(const int32_t *xy, int64_t n, const int32_t *t, int64_t i, int64_t o)
{
    const int64_t j = (i + o) % n;
    const int64_t a = t[i], b = t[(i + 1) % n], c = t[j], e = t[(j + 1) % n];
    return oracle_dist(xy, a, c) + oracle_dist(xy, b, e) - oracle_dist(xy, a, b) -
           oracle_dist(xy, c, e);
}

/* best move of every position: off[i] = 0 when no move has g < 0 */
void oracle_two_opt_best(const int32_t *xy, int64_t n, const int32_t *tour, int64_t window,
                         int64_t *gain, int64_t *off)
{
    const int64_t W = two_opt_window(n, window);
    for (int64_t i = 0; i < n; ++i) {
        gain[i] = 0;
        off[i] = 0;
        for (int64_t o = 2; o <= W; ++o) {
            const int64_t g = two_opt_gain(xy, n, tour, i, o);
            if (g < gain[i]) {
                gain[i] = g;
                off[i] = o;
            }
        }
    }
}

/* Runs rounds until none improves or max_rounds (> 0) rounds have     */
/* applied moves.  Returns the rounds that applied moves; *moves the    */
/* moves, *gain their summed gains, *converged 1 when the last round    */
/* found no improving move.                                             */
int64_t oracle_two_opt(const int32_t *xy, int64_t n, int32_t *tour, int64_t window,
                       int64_t max_rounds, int64_t *moves, int64_t *gain, int *converged)
{
    *moves = 0;
    *gain = 0;
    *converged = 1;
    const int64_t W = two_opt_window(n, window);
    if (W < 2) return 0;
    int64_t *g = malloc((size_t)n * sizeof *g);
    int64_t *o = malloc((size_t)n * sizeof *o);
    uint8_t *take = malloc((size_t)n);
    int64_t *cand = malloc((size_t)n * sizeof *cand);
    int64_t rounds = 0;
    for (;;) {
        oracle_two_opt_best(xy, n, tour, window, g, o);
        int64_t nc = 0;   /* positions with an improving move */
        for (int64_t i = 0; i < n; ++i)
            if (o[i] != 0) cand[nc++] = i;
        if (nc == 0) break;
        if (max_rounds > 0 && rounds == max_rounds) {
            *converged = 0;
            break;
        }
        /* choose: no overlapping move is better by (g, position) */
        for (int64_t i = 0; i < n; ++i) {
            take[i] = o[i] != 0;
            for (int64_t x = 0; x < nc && take[i]; ++x) {
                const int64_t u = cand[x];
                if (u == i) continue;
                /* spans [i, i+o[i]+1] and [u, u+o[u]+1] overlap (cyclic)? */
                const int64_t du = (u - i + n) % n;   /* u's distance ahead of i */
                const int64_t di = (i - u + n) % n;   /* i's distance ahead of u */
                const int overlap = du <= o[i] + 1 || di <= o[u] + 1;
                if (overlap && (g[u] < g[i] || (g[u] == g[i] && u < i))) take[i] = 0;
            }
        }
        for (int64_t i = 0; i < n; ++i) {
            if (!take[i]) continue;
            for (int64_t q = 0; q < o[i] / 2; ++q) {
                const int64_t p1 = (i + 1 + q) % n, p2 = (i + o[i] - q) % n;
                const int32_t tmp = tour[p1];
                tour[p1] = tour[p2];
                tour[p2] = tmp;
            }
            *moves += 1;
            *gain += g[i];
        }
        ++rounds;
    }
    free(g);
    free(o);
    free(take);
    free(cand);
    return rounds;
}

/* ------------------------------------------------------------------ */
/* Pheromone update: evaporation (Eq. 2) then the deposit of every ant  */
/* (Eq. 3-4), Delta tau = 1/C^k on the edges of ant k's tour, quantised  */
/* to int64 fixed point q = floor(2^shift / L) and accumulated exactly. */
/* Each undirected edge {i,j} is stored as up to two directed slots      */
/* (j in nn[i], i in nn[j]); both get the deposit, absent slots nothing. */
/* ------------------------------------------------------------------ */

/* acc = sum over tours a of q[a] on both directed slots of every tour edge */
static void deposit_quanta(int64_t n, int k, const int32_t *nn, int64_t m, const int32_t *tours,
                           const int64_t *qa, int64_t *acc)
{
    memset(acc, 0, (size_t)(n * k) * sizeof(int64_t));
    for (int64_t a = 0; a < m; a++) {
        int64_t q = qa[a];
        const int32_t *T = tours + a * n;
        for (int64_t t = 0; t < n; t++) {
            int64_t i = T[t], j = T[(t + 1) % n];
            for (int r = 0; r < k; r++)
                if (nn[i * k + r] == j) acc[i * k + r] += q;
            for (int r = 0; r < k; r++)
                if (nn[j * k + r] == i) acc[j * k + r] += q;
        }
    }
}

/* The deposit of ants a0..a1-1 into acc (zeroed first). */
static void deposit_ants(int64_t n, int k, const int32_t *nn, int64_t a0, int64_t a1,
                         const int32_t *tours, const int64_t *lengths, int shift, int64_t *acc)
{
    memset(acc, 0, (size_t)(n * k) * sizeof(int64_t));
    for (int64_t a = a0; a < a1; a++) {
        int64_t q = ((int64_t)1 << shift) / lengths[a];
        const int32_t *T = tours + a * n;
        for (int64_t t = 0; t < n; t++) {
            int64_t i = T[t], j = T[(t + 1) % n];
            for (int r = 0; r < k; r++)
                if (nn[i * k + r] == j) acc[i * k + r] += q;
            for (int r = 0; r < k; r++)
                if (nn[j * k + r] == i) acc[j * k + r] += q;
        }
    }
}

typedef struct {
    int64_t n; int k; const int32_t *nn; int64_t a0, a1;
    const int32_t *tours; const int64_t *lengths; int shift; int64_t *acc;
} deposit_job_t;

static void *deposit_worker(void *arg)
{
    deposit_job_t *J = (deposit_job_t *)arg;
    deposit_ants(J->n, J->k, J->nn, J->a0, J->a1, J->tours, J->lengths, J->shift, J->acc);
    return NULL;
}

/* Threads take contiguous groups of ants into private sums, added at the end:
 * integer addition, so the result does not depend on the split. */
void oracle_deposit(int64_t n, int k, const int32_t *nn, int64_t m, const int32_t *tours,
                    const int64_t *lengths, int shift, int64_t *acc, int threads)
{
    if (threads > m) threads = (int)m;
    if (threads > 64) threads = 64;
    if (threads <= 1) {
        deposit_ants(n, k, nn, 0, m, tours, lengths, shift, acc);
        return;
    }
    deposit_job_t job[64];
    pthread_t th[64];
    for (int t = 0; t < threads; t++) {
        job[t] = (deposit_job_t){n, k, nn, m * t / threads, m * (t + 1) / threads, tours, lengths,
                                 shift, t == 0 ? acc : (int64_t *)malloc((size_t)(n * k) * 8)};
        pthread_create(&th[t], NULL, deposit_worker, &job[t]);
    }
    for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
    for (int t = 1; t < threads; t++) {
        for (int64_t e = 0; e < n * k; e++) acc[e] += job[t].acc[e];
        free(job[t].acc);
    }
}

void oracle_update(int64_t n, int k, const int32_t *nn, float *tau, int64_t m, const int32_t *tours,
                   const int64_t *lengths, double rho, int shift, int threads)
{
    int64_t *acc = (int64_t *)malloc((size_t)(n * k) * sizeof(int64_t));
    oracle_deposit(n, k, nn, m, tours, lengths, shift, acc, threads);
    float f = (float)(1.0 - rho);
    float scale = ldexpf(1.0f, -shift);
    for (int64_t e = 0; e < n * k; e++) {
        float evap = tau[e] * f;                       /* Eq. 2, FP32 */
        float dep = (float)acc[e] * scale;             /* exact power-of-two scaling */
        tau[e] = evap + dep;                           /* Eq. 3, one FP32 rounding */
    }
    free(acc);
}

/* ------------------------------------------------------------------ */
/* Construction of many ants, threads over ants.                        */
/* ------------------------------------------------------------------ */

typedef struct {
    const colony_t *C;
    const int64_t *ants;
    int64_t count;
    int32_t *tours;
    int64_t *lengths;
    int8_t *slots;
    double *probs;
    int64_t *fallbacks;
    int64_t next;
    pthread_mutex_t lock;
} pool_t;

static void *construct_worker(void *arg)
{
    pool_t *P = (pool_t *)arg;
    int64_t n = P->C->n;
    for (;;) {
        pthread_mutex_lock(&P->lock);
        int64_t q = P->next++;
        pthread_mutex_unlock(&P->lock);
        if (q >= P->count) break;
        ant_result_t r = construct_ant(P->C, P->ants[q], P->tours + q * n,
                                       P->slots ? P->slots + q * n : NULL,
                                       P->probs ? P->probs + q * n : NULL);
        P->lengths[q] = r.length;
        if (P->fallbacks) P->fallbacks[q] = r.fallbacks;
    }
    return NULL;
}

static void colony_init(colony_t *C, int64_t n, int k, const int32_t *xy, const int32_t *nn,
                        const int32_t *nnd, const float *tau, const double *eta, double alpha,
                        double beta, uint64_t seed, int64_t iteration)
{
    C->n = n; C->k = k; C->xy = xy; C->nn = nn; C->nnd = nnd; C->tau = tau; C->eta = eta;
    C->alpha = alpha; C->beta = beta; C->seed = seed; C->iteration = iteration;
    C->sampler = 0;
    C->xorder = NULL;
    C->xpos = NULL;
}

/* Construct the ants listed in `ants` (count of them); outputs are [count][n]. */
void oracle_construct(int64_t n, int k, const int32_t *xy, const int32_t *nn, const int32_t *nnd,
                      const float *tau, const double *eta, double alpha, double beta, uint64_t seed,
                      int64_t iteration, const int64_t *ants, int64_t count, int32_t *tours,
                      int64_t *lengths, int8_t *slots, double *probs, int64_t *fallbacks,
                      int threads)
{
    colony_t C;
    colony_init(&C, n, k, xy, nn, nnd, tau, eta, alpha, beta, seed, iteration);
    pool_t P = {&C, ants, count, tours, lengths, slots, probs, fallbacks, 0,
                PTHREAD_MUTEX_INITIALIZER};
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    for (int t = 0; t < threads; t++) pthread_create(&th[t], NULL, construct_worker, &P);
    for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
}

void oracle_replay(int64_t n, int k, const int32_t *xy, const int32_t *nn, const int32_t *nnd,
                   const float *tau, const double *eta, double alpha, double beta, uint64_t seed,
                   int64_t iteration, int64_t ant, const int32_t *tour, double boundary_eps,
                   const int32_t *xorder, const int32_t *xpos, double *prob, int64_t *out)
{
    colony_t C;
    colony_init(&C, n, k, xy, nn, nnd, tau, eta, alpha, beta, seed, iteration);
    C.xorder = xorder;
    C.xpos = xpos;
    oracle_replay_ant(&C, ant, tour, boundary_eps, prob, out);
}

/* ------------------------------------------------------------------ */
/* The whole loop for one instance: candidates, NN-tour initialisation, */
/* then `iterations` rounds of construction and update.  The iteration  */
/* best is the shortest tour (lowest ant on ties); the global best is   */
/* replaced only by a strictly shorter tour.                            */
/* ------------------------------------------------------------------ */

int oracle_run(int64_t n, int k, const int32_t *xy, int64_t m, double alpha, double beta, double rho,
               int64_t iterations, uint64_t seed, int shift, int threads, int32_t *best_tour,
               int64_t *best_len, int64_t *iter_best, float *tau_out)
{
    int32_t *nn = (int32_t *)malloc((size_t)(n * k) * 4);
    int32_t *nnd = (int32_t *)malloc((size_t)(n * k) * 4);
    int32_t *rows = (int32_t *)malloc((size_t)n * 4);
    float *tau = (float *)malloc((size_t)(n * k) * 4);
    int32_t *tours = (int32_t *)malloc((size_t)(m * n) * 4);
    int64_t *lengths = (int64_t *)malloc((size_t)m * 8);
    int64_t *ants = (int64_t *)malloc((size_t)m * 8);
    for (int64_t i = 0; i < n; i++) rows[i] = (int32_t)i;
    oracle_knn_rows(xy, n, k, rows, n, nn, nnd);
    int64_t Lnn = oracle_nn_tour(xy, n, k, nn, nnd, best_tour);
    if (Lnn <= 0) {
        free(nn); free(nnd); free(rows); free(tau); free(tours); free(lengths); free(ants);
        return -3;   /* every city coincident: tau0 undefined */
    }
    *best_len = Lnn;   /* best so far starts as the NN tour */
    float t0 = oracle_tau0(n, Lnn);
    for (int64_t e = 0; e < n * k; e++) tau[e] = t0;
    for (int64_t a = 0; a < m; a++) ants[a] = a;
    for (int64_t it = 0; it < iterations; it++) {
        oracle_construct(n, k, xy, nn, nnd, tau, NULL, alpha, beta, seed, it, ants, m, tours,
                         lengths, NULL, NULL, NULL, threads);
        int64_t ib = 0;
        for (int64_t a = 1; a < m; a++)
            if (lengths[a] < lengths[ib]) ib = a;
        if (iter_best) iter_best[it] = lengths[ib];
        if (lengths[ib] < *best_len) {
            *best_len = lengths[ib];
            memcpy(best_tour, tours + ib * n, (size_t)n * 4);
        }
        oracle_update(n, k, nn, tau, m, tours, lengths, rho, shift, threads);
    }
    if (tau_out) memcpy(tau_out, tau, (size_t)(n * k) * 4);
    free(nn); free(nnd); free(rows); free(tau); free(tours); free(lengths); free(ants);
    return 0;
}
