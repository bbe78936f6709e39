/*
 * aco.h -- C ABI of the MI355X ACO hot-path library (libaco.so).
 *
 * Ant colony optimisation for the symmetric TSP (Chitty, "Applying ACO To
 * Large Scale TSP Instances", Section 2): m ants build tours with the random
 * proportional rule (Eq. 1), then the pheromone is evaporated (Eq. 2) and
 * every ant deposits 1/C^k on the edges of its tour (Eq. 3-4).  Pheromone is
 * held only on each city's k nearest-neighbour candidate edges (an n x k
 * table instead of the n x n matrix whose size Section 3 identifies as the
 * obstacle to large instances; candidate lists are the ACS device recalled in
 * Section 6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array arguments are DEVICE pointers into memory owned by the caller
 *   (e.g. torch tensors); host pointers are marked "host".  Row-major layouts,
 *   no padding.  The library keeps no pointer after a call returns, but the
 *   work it enqueued reads and writes the buffers until the stream reaches it.
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  All work is
 *   enqueued on it in order; entry points marked "synchronises" wait for it.
 * - Return value: ACO_OK (0) or a negative ACO_ERR_* code.  Arguments are
 *   validated on the host before anything is enqueued: on a validation error
 *   nothing is launched and the outputs are untouched.  aco_last_error()
 *   returns a thread-local message for the most recent failure.
 * - Cities are numbered 0..n-1 in input order; "index" always means that
 *   number.  Distances are d_ij = nint(sqrt((xi-xj)^2 + (yi-yj)^2)) (Section
 *   2 requires only d_ij = d_ji; the rounded Euclidean form is the TSPLIB
 *   EUC_2D convention), computed exactly in integers.
 * - Coordinates must satisfy |x|, |y| <= ACO_COORD_LIMIT.
 * - Random numbers: Philox4x32-10 with key (seed low 32 bits, seed high 32
 *   bits) and counter (step, ant, iteration, 0); word 0 is used.  Step 0 draws
 *   the start city (x * n) >> 32 (Section 2: ants start at a random city);
 *   step t >= 1 draws u = x * 2^-32 for the roulette of Eq. 1.
 */
#ifndef ACO_H
#define ACO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ACO_OK 0
#define ACO_ERR_INVALID_ARG (-1) /* a size, pointer or parameter is out of range */
#define ACO_ERR_UNSUPPORTED (-2) /* valid, but beyond what the library supports (e.g. LDS) */
#define ACO_ERR_DEGENERATE (-3)  /* every city coincides: the NN tour has length 0 */
#define ACO_ERR_WORKSPACE (-4)   /* workspace smaller than the matching *_bytes query */
#define ACO_ERR_HIP (-5)         /* a HIP runtime call failed */
#define ACO_ERR_DEVICE (-6)      /* a kernel found device data breaking a stated precondition */

#define ACO_COORD_LIMIT 536870911 /* 2^29 - 1: every distance fits in int32 */
#define ACO_MAX_K 64               /* one candidate per lane of a 64-wide wavefront */

/* Human-readable name of an ACO_* code (static string). */
const char *aco_strerror(int code);
/* Message describing the last failure on the calling thread ("" if none). */
const char *aco_last_error(void);
/* Library version string. */
const char *aco_version(void);

/* Device-side checks.  Some preconditions depend on device data the host does
 * not read before a launch (a local best that is not a permutation, a tour
 * entry out of range, a tour length <= 0, ...).  A kernel
 * that meets one keeps every access in range, finishes normally and sets a
 * bit in the current device's error word (one word per device, shared by all
 * streams and threads).  Every entry point that synchronises reports and
 * clears it after its own work: ACO_ERR_DEVICE, with aco_last_error() naming
 * the checks that failed.  Results written since the first failure are not
 * to be trusted.
 *
 * aco_device_error: synchronises with `stream` and reports the word as
 * above (ACO_OK when no check failed since the last report).  Errors: DEVICE,
 * HIP. */
int aco_device_error(void *stream);

/* One query for the workspace of any entry point that takes one (each also
 * has its own query below):
 *   ACO_WS_GRID        aco_grid_bytes(n)
 *   ACO_WS_CONSTRUCT   aco_construct_workspace_bytes(n, k)
 *   ACO_WS_UPDATE      aco_update_workspace_bytes(n, k, m)
 *   ACO_WS_RUN         aco_run_workspace_bytes(n, {m, k, eta = 1/d})
 *   ACO_WS_TWO_OPT     aco_two_opt_workspace_bytes(n, m, 1)
 *   ACO_WS_FEATURES    aco_features_workspace_bytes()
 *   ACO_WS_MLP_BACKWARD aco_mlp_backward_workspace_bytes(n * k edges)
 * Returns 0 for an unknown `which` or sizes the query refuses.  (The batched
 * workspace depends on every instance's size: aco_batch_workspace_bytes.) */
#define ACO_WS_GRID 0
#define ACO_WS_CONSTRUCT 1
#define ACO_WS_UPDATE 2
#define ACO_WS_RUN 3
#define ACO_WS_TWO_OPT 4
#define ACO_WS_FEATURES 5
#define ACO_WS_MLP_BACKWARD 6
size_t aco_workspace_bytes(int32_t which, int32_t n, int32_t k, int32_t m);

/* ------------------------------------------------------------------------
 * Candidate lists and spatial grid.
 *
 * For every city i: nn[i][r], r = 0..k-1, are the k cities j != i with the
 * smallest keys (d_ij, j), ascending (distance, then index); nnd[i][r] =
 * d_{i,nn[i][r]}; rev[i][r] = the position of i in nn[nn[i][r]] or -1;
 * eta_b[i][r] = eta^beta rounded once to FP32, with eta = 1/max(d, 1) (Section
 * 2: eta_ij = 1/d_ij; coincident cities read as d = 1) or, when `eta` is not
 * NULL, eta = eta[i][r] (a learned heuristic score > 0, FP32 [n][k]).
 *
 * The grid (uniform square cells, about two cities per cell) serves the
 * nearest-unvisited fallback.  It is an opaque device buffer of
 * aco_grid_bytes(n) bytes written here and read by the other entry points.
 *
 *   xy     int32 [n][2]   coordinates (x, y)
 *   n      3 <= n <= 2^27;  k: 1 <= k <= min(n-1, ACO_MAX_K);  beta >= 0, finite
 *   nn, nnd int32 [n][k]; rev int8 [n][k]; eta_b float [n][k]   (outputs)
 * Synchronises (reads back the bounding box to size the grid).
 * Errors: INVALID_ARG (sizes, NULL pointers, |coord| > ACO_COORD_LIMIT),
 *         DEGENERATE (all cities coincide), WORKSPACE (grid_bytes too small).
 * ------------------------------------------------------------------------ */
size_t aco_grid_bytes(int32_t n);
int aco_build_candidates(const int32_t *xy, int32_t n, int32_t k, double beta, const float *eta,
                         int32_t *nn, int32_t *nnd, int8_t *rev, float *eta_b, void *grid,
                         size_t grid_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Pheromone initialisation: the nearest-neighbour tour from city 0 (each step
 * takes the unvisited city of smallest (d, j)), its length L_nn, and
 * tau[i][r] = tau0 = fl32(1 / (n * L_nn)) for every candidate slot.
 *
 *   grid      the buffer from aco_build_candidates (8 bytes of its header
 *             block are used as scratch for the tour length)
 *   nn_tour   int32 [n] (output)   tau float [n][k] (output)
 *   tau0_out  host float* (output, may be NULL); L_nn_out host int64* (may be NULL)
 * The tour takes two steps per table row where it can, from a table of 256
 * bytes per city held in stream-ordered scratch (hipMallocAsync on `stream`,
 * freed before the call returns; HIP error if it cannot be had).
 * Synchronises (and reports device checks, see aco_device_error).
 * Errors: INVALID_ARG, DEGENERATE (L_nn == 0), UNSUPPORTED (visited bitmask
 * of ceil(n/32) words does not fit in LDS), DEVICE.
 * ------------------------------------------------------------------------ */
int aco_init_pheromone(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                       const int32_t *nnd, void *grid, int32_t *nn_tour, float *tau,
                       float *tau0_out, int64_t *L_nn_out, void *stream);

/* ------------------------------------------------------------------------
 * Tour construction (Section 2, Eq. 1).  Ant a (0 <= a < m) starts at
 * (x * n) >> 32 and at every later step, standing at city c, considers the
 * unvisited candidates r of c in rank order with weights
 *     w_r = tau[c][r]^alpha * eta_b[c][r]
 * and moves to the first r with u * S < C_r, S the total weight and C_r the
 * running sum (a zero-weight candidate is never chosen).  When no unvisited
 * candidate has positive weight the ant moves to the nearest unvisited city
 * (smallest (d, j)), found exactly on the grid.
 *
 *   nn, nnd, eta_b, grid   as written by aco_build_candidates (eta_b possibly
 *            replaced by a learned table); the kernels take the candidate
 *            lists from the grid's table by position, which holds the same
 *            lists as nn, so nn must be the lists this grid was built with
 *   tau      float [n][k]  pheromone (read)
 *   ant0     index of the first ant (ants ant0..ant0+m-1 are built; the
 *            Philox counter uses the absolute ant index)
 *   tours    int32 [m][n]  (output) city order, tours[a][0] = start city
 *   lengths  int64 [m]     (output) closed tour length C^a
 *   slots    uint8 [m][n]  (output) slots[a][t] = rank r of tours[a][t] in
 *            nn[tours[a][t-1]], 255 for a fallback move; slots[a][0] = 255
 *   step_prob float [m][n] (output, may be NULL) probability of the move
 *            taken at step t (-1 for a fallback move; 1 at t = 0)
 *   ws       device workspace of aco_construct_workspace_bytes(n, k) bytes
 *            (the choice rows: n rows of 16, 32 or 64 elements of 8 bytes
 *            for k <= 16, <= 32, <= 64, so that each row starts on a
 *            128-byte line)
 * Constraints: 0 <= iteration < 2^32, m >= 1, alpha >= 0 finite.
 * Errors: INVALID_ARG, WORKSPACE, UNSUPPORTED (bitmask does not fit in LDS).
 * ------------------------------------------------------------------------ */
size_t aco_construct_workspace_bytes(int32_t n, int32_t k);
int aco_construct_tours(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                        const int32_t *nnd, const float *eta_b, const void *grid, const float *tau,
                        int32_t m, int32_t ant0, double alpha, uint64_t seed, int64_t iteration,
                        int32_t *tours, int64_t *lengths, uint8_t *slots, float *step_prob,
                        void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Pheromone update.  Evaporation tau' = fl32(tau * fl32(1 - rho)) on every
 * candidate slot (Eq. 2), then the deposit of every ant (Eq. 3-4): ant a adds
 * q_a = floor(2^deposit_shift / lengths[a]) (1/C^a in fixed point) to each
 * directed slot (i, r) with nn[i][r] = j for every edge {i, j} of its tour,
 * the closing edge included, in both directions when both slots exist; edges
 * outside the candidate lists carry no pheromone.  Sums are exact in int64,
 * and the merge is tau = fl32(tau' + fl32(acc) * 2^-deposit_shift).
 *
 *   tours int32 [m][n] (any permutations), slots uint8 [m][n]: the record
 *   aco_construct_tours wrote for exactly these tours (trusted: a record of
 *   other tours gives wrong pheromone, unreported; checking it would cost a
 *   gather per edge), or NULL (then every edge is located by scanning the
 *   candidate rows), lengths int64 [m] > 0,
 *   0 < rho <= 1, 0 <= deposit_shift <= 62 (m * floor(2^shift / L) < 2^63
 *   for every length L keeps the int64 sums exact),
 *   tau float [n][k] (in/out), ws: aco_update_workspace_bytes(n, k, m) bytes.
 * Errors: INVALID_ARG, WORKSPACE.  Device checks (ACO_ERR_DEVICE, see
 * aco_device_error): a tour entry out of range (that edge is skipped), a
 * length <= 0 (its deposit is 0) or a quantum with m * q >= 2^63.
 * ------------------------------------------------------------------------ */
size_t aco_update_workspace_bytes(int32_t n, int32_t k, int32_t m);
int aco_update_pheromone(int32_t n, int32_t k, const int32_t *nn, const int8_t *rev, int32_t m,
                         const int32_t *tours, const uint8_t *slots, const int64_t *lengths,
                         double rho, int32_t deposit_shift, float *tau, void *ws, size_t ws_bytes,
                         void *stream);

/* The same update without a workspace argument, for callers that cannot
 * allocate device memory (code being captured into a HIP graph, serving
 * loops, harnesses that forbid allocation).  It allocates nothing: the slot
 * sums and quanta live in a scratch array the library holds on every device
 * it runs on (ACO_UPDATE_STATIC_BYTES bytes each, kept until the process
 * ends), so aco_update_workspace_bytes(n, k, m) must not exceed
 * ACO_UPDATE_STATIC_BYTES (n = 200,000 and k = 16 fit with m up to
 * 994,000).  The scratch is cleared by a kernel at the start of every call.
 * Calls on one device share that scratch: two calls that overlap (on
 * different streams, or from different threads without ordering) race and
 * give wrong pheromone.  Results are bit-identical to aco_update_pheromone's.
 * Errors: INVALID_ARG (as aco_update_pheromone, and sizes beyond the
 * scratch), HIP.  Device checks as aco_update_pheromone. */
#define ACO_UPDATE_STATIC_BYTES (32u << 20)
int aco_update_pheromone_static(int32_t n, int32_t k, const int32_t *nn, const int8_t *rev,
                                int32_t m, const int32_t *tours, const uint8_t *slots,
                                const int64_t *lengths, double rho, int32_t deposit_shift,
                                float *tau, void *stream);

/* ------------------------------------------------------------------------
 * Best-tour tracking (the method outputs the best tour found, Alg. 1's last
 * step).  The iteration best is the shortest of lengths[0..m) (lowest ant on
 * ties); it replaces the best so far only when strictly shorter.
 *
 *   best_len   int64 [1] (in/out, device)   best_tour int32 [n] (in/out)
 *   iter_best  int64 [1] (output, device; may be NULL)
 * ------------------------------------------------------------------------ */
int aco_track_best(int32_t n, int32_t m, const int32_t *tours, const int64_t *lengths,
                   int64_t *best_len, int32_t *best_tour, int64_t *iter_best, void *stream);

/* ------------------------------------------------------------------------
 * The whole loop on one instance: candidates, NN-tour initialisation (the
 * best so far starts as the NN tour), then `iterations` rounds of
 * construction (iteration t uses the pheromone after t updates), update and
 * best tracking.
 * ------------------------------------------------------------------------ */
#define ACO_ETA_DISTANCE 0 /* eta = 1/d (Section 2) */
#define ACO_ETA_LEARNED 1  /* eta = sigmoid of the edge-scoring network's score (below) */

typedef struct aco_params {
    uint32_t struct_size;  /* sizeof(aco_params_t) as the caller was built (see below) */
    int32_t m;             /* ants per iteration, >= 1 */
    int32_t k;             /* candidates per city (0: k-auto, aco_run_batched only) */
    double alpha;          /* pheromone exponent, >= 0 */
    double beta;           /* heuristic exponent, >= 0 */
    double rho;            /* evaporation rate, 0 < rho <= 1 */
    int32_t iterations;    /* >= 0 */
    int32_t deposit_shift; /* fixed-point fraction bits of the deposit, 0..62 (32) */
    uint64_t seed;         /* Philox key */
    int32_t eta_mode;      /* ACO_ETA_DISTANCE (default) or ACO_ETA_LEARNED (aco_run only) */
    const float *mlp_w;    /* ACO_ETA_LEARNED: device FP32 [ACO_MLP_PARAMS] network parameters */
} aco_params_t;
/* The library reads only the caller's struct_size bytes; later fields take
 * their defaults (eta_mode ACO_ETA_DISTANCE, mlp_w NULL).  struct_size must
 * cover the fields through seed (INVALID_ARG otherwise).  The batched entry
 * points refuse ACO_ETA_LEARNED (UNSUPPORTED). */

size_t aco_run_workspace_bytes(int32_t n, const aco_params_t *p);
/*   best_tour int32 [n], best_len int64 [1] (outputs, device)
 *   iter_best int64 [iterations] (output, may be NULL)
 *   tau_out   float [n][k] final pheromone (output, may be NULL)
 * With ACO_ETA_LEARNED the candidate edges' features (aco_edge_features) go
 * through the network (aco_mlp_forward) right after the candidate build, and
 * eta_b = sigmoid(z)^beta replaces (1/d)^beta; the workspace then also holds
 * the features (32 bytes per candidate slot).
 * Synchronises (during set-up).  Errors: as the steps above; INVALID_ARG for
 * an unknown eta_mode or ACO_ETA_LEARNED without mlp_w. */
int aco_run(const int32_t *xy, int32_t n, const aco_params_t *p, int32_t *best_tour,
            int64_t *best_len, int64_t *iter_best, float *tau_out, void *ws, size_t ws_bytes,
            void *stream);

/* ------------------------------------------------------------------------
 * Batched colonies: B independent instances of uneven size, each running the
 * loop of aco_run (same rules, same Philox keying with the ant index local to
 * its instance), concatenated in CSR form.
 *
 *   xy        int32 [N][2], N = offsets[B]; instance b owns rows
 *             offsets[b] .. offsets[b+1]-1 and numbers its cities from 0
 *   offsets   HOST int64 [B+1], offsets[0] = 0; every n_b >= 3, n_b <= 65536,
 *             k <= min over b of n_b - 1; 1 <= m <= 1024
 *   best_tours int32 [N]  (output) best tour of each instance, local indices
 *   best_lens  int64 [B]  (output)
 *   iter_best  int64 [B][iterations] (output, may be NULL)
 *   ws         device workspace of aco_batch_workspace_bytes(offsets, B, p)
 *
 * aco_batch_setup builds every instance's grid, candidate lists and
 * nearest-neighbour tour (the best so far starts as that tour) and
 * synchronises to report INVALID_ARG / DEGENERATE (and device checks, see
 * aco_device_error).  aco_batch_iterate then
 * runs iterations first .. first+count-1 of every instance in ONE persistent
 * kernel launch (no allocation, no host synchronisation: it can be captured in
 * a HIP graph); its iter_best is [B][count].  `waves` = waves per instance
 * workgroup (1, 2, 4, 8, 16), `vis_layout` = ACO_VIS_BITS / ACO_VIS_BYTES (one
 * ant per wave, a bit or a byte per city) or ACO_VIS_BITS_X4 (four ants per
 * wave on its four 16-lane rows, a bit per city each; k <= 16) and
 * `occupancy` = waves per SIMD the kernel's registers allow (4 or 8), each 0
 * for the tuned value (before tuning: four ants per wave with the most waves
 * the LDS holds when k <= 16, else 8 waves, bits, 4 per SIMD), change the
 * speed, never the results.  aco_run_batched
 * = set-up + all iterations.  With autotune != 0 every candidate shape runs
 * iteration 0 from the state the set-up left (restored before each, timed),
 * then the state is restored and all iterations run in the fastest shape
 * (cached per device and shape; the results equal those of any fixed shape).
 * With p->k == 0 (k-auto, aco_run_batched only) the candidate counts 8, 10,
 * 12 and 16 (those <= min n_b - 1) each run the set-up and min(iterations, 8)
 * iterations; a candidate's quality after i iterations is the mean over
 * instances of best-so-far / NN-tour length; the target is the worst final
 * quality among them, and the k that reaches it in the least time (iterations
 * times its time per iteration; ties to the smaller k) is set up afresh and
 * runs all iterations.  tuned_out (host int32 [4], may be NULL) receives
 * {waves, layout, occupancy, k}.  The tuning steps allocate stream-ordered
 * scratch (hipMallocAsync) and free it before the run.
 * aco_batch_workspace_bytes with k = 0 sizes for the largest candidate.
 * step_prob (aco_batch_iterate; float, laid out as the tours, may be NULL)
 * receives the probability of every move of the last iteration run, as
 * aco_construct_tours' step_prob; it needs one ant per wave (an explicit
 * ACO_VIS_BITS_X4 is refused, the default shape falls back to bits).
 * aco_batch_layout gives the byte offsets of the state arrays inside ws
 * (for inspection: nn/nnd/rev/eta_b/tau are [N][k], tours/slots are instance
 * b at m*offsets[b] as [m][n_b], lengths [B][m]).
 * ------------------------------------------------------------------------ */
#define ACO_VIS_BITS 1
#define ACO_VIS_BYTES 2
#define ACO_VIS_BITS_X4 3

typedef struct aco_batch_layout {
    size_t nn, nnd, rev, eta_b, tau, tours, slots, lengths, total;
} aco_batch_layout_t;

size_t aco_batch_workspace_bytes(const int64_t *offsets, int32_t B, const aco_params_t *p);
int aco_batch_layout(const int64_t *offsets, int32_t B, const aco_params_t *p,
                     aco_batch_layout_t *out);
int aco_batch_setup(const int32_t *xy, const int64_t *offsets, int32_t B, const aco_params_t *p,
                    int32_t *best_tours, int64_t *best_lens, void *ws, size_t ws_bytes,
                    void *stream);
int aco_batch_iterate(const int32_t *xy, const int64_t *offsets, int32_t B,
                      const aco_params_t *p, int32_t first_iteration, int32_t count,
                      int32_t waves, int32_t vis_layout, int32_t occupancy, int32_t *best_tours,
                      int64_t *best_lens, int64_t *iter_best, float *step_prob, void *ws,
                      size_t ws_bytes, void *stream);
int aco_run_batched(const int32_t *xy, const int64_t *offsets, int32_t B, const aco_params_t *p,
                    int32_t autotune, int32_t *best_tours, int64_t *best_lens,
                    int64_t *iter_best, void *ws, size_t ws_bytes, void *stream,
                    int32_t *tuned_out);

/* ------------------------------------------------------------------------
 * PartialACO (Section 3.1, Algorithm 1).  Each ant keeps part of its own
 * best tour so far (its local best) and rebuilds only the rest with the rule
 * of Eq. 1; Section 4 caps the rebuilt share and lets an ant build a full
 * tour with probability 1 - p.  The plan of ant a at an iteration comes from
 * the Philox block at counter (0, a, iteration): word 0 gives the start
 * position s = (x0 n) >> 32 in the local best tour, word 1 the partial
 * decision x1 < round(p 2^32), word 2 the rebuilt count
 * r = 1 + ((x2 M) >> 32), uniform on [1, M] with M = max_modify clamped to
 * [1, n-1].  A partial tour is lbest[s], ..., lbest[s + n - r - 1] (cyclic)
 * followed by r cities constructed from the last kept city; tour position t
 * draws from counter (t, a, iteration) as in aco_construct_tours, so an ant
 * that builds a full tour (and p = 0) gives exactly aco_construct_tours'
 * tour.  Kept positions carry slot 255 (no construction record) and step_prob 1.
 * Iteration 0 is a full construction; the local bests start as its tours.
 * ------------------------------------------------------------------------ */

/* As aco_construct_tours, plus:
 *   p_partial   probability in [0, 1] that an ant only partially rebuilds
 *   max_modify  cap M >= 1 on the rebuilt cities (the paper uses 1% at 200K)
 *   lbest       int32 [m][n] the ants' local best tours (city indices; row a
 *               for ant ant0 + a), read only
 * Errors: as aco_construct_tours; INVALID_ARG for lbest NULL, p outside
 * [0, 1], max_modify < 1.  lbest rows must be permutations of 0..n-1. */
int aco_construct_partial(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                          const int32_t *nnd, const float *eta_b, const void *grid,
                          const float *tau, int32_t m, int32_t ant0, double alpha, uint64_t seed,
                          int64_t iteration, double p_partial, int32_t max_modify,
                          const int32_t *lbest, int32_t *tours, int64_t *lengths, uint8_t *slots,
                          float *step_prob, void *ws, size_t ws_bytes, void *stream);

/* Construction with options: the sampler of the next city and PartialACO.
 *   sampler ACO_SAMPLER_ROULETTE: Eq. 1 as in aco_construct_tours;
 *           ACO_SAMPLER_INDEPENDENT: Independent Roulette (Section 3): among
 *           the unvisited candidates with positive weight the largest
 *           w_r * U_r (FP64) wins, ties to the lower rank; U_r = x * 2^-32 with
 *           x word (r mod 4) of the Philox block at counter
 *           (t, ant, iteration, 1 + r / 4).  Its move probabilities are not
 *           computed: step_prob must be NULL.
 *   lbest   NULL for full tours, else PartialACO with p_partial and
 *           max_modify as in aco_construct_partial.
 *   lbest_len  NULL, or device int64 [m] with the exact closed length of
 *           every local best (as aco_update_local_best keeps it): the kept
 *           part's length is then that length minus the edges outside the
 *           kept part, instead of a sum over the kept part (same result when
 *           the lengths are exact).  A length that no tour of n cities can
 *           have (<= 0, or >= n 2^31, such as the INT64_MAX start value) trips
 *           a device check (ACO_ERR_DEVICE) and that ant's kept part is
 *           summed edge by edge; so does a result that comes out <= 0.  Any
 *           other wrong length gives a wrong tour length, unreported.
 *   Device checks (ACO_ERR_DEVICE, see aco_device_error): an lbest row that
 *   is not a permutation of 0..n-1 (out-of-range entries are read as city 0).
 * opts is a host pointer (NULL: roulette, full tours).  Other arguments and
 * errors as aco_construct_tours; Independent Roulette also keeps one block of
 * uniforms in LDS (64 steps x k rounded up to 4 words), so UNSUPPORTED is
 * returned when that and the visited bitmask together do not fit. */
#define ACO_SAMPLER_ROULETTE 0
#define ACO_SAMPLER_INDEPENDENT 1
typedef struct aco_construct_opts {
    uint32_t struct_size;       /* sizeof(aco_construct_opts_t) as the caller was built */
    int32_t sampler;
    double p_partial;
    int32_t max_modify;
    const int32_t *lbest;
    const int64_t *lbest_len;   /* [m] or NULL (see above) */
} aco_construct_opts_t;
/* struct_size lets the struct grow: the library reads only the caller's
 * struct_size bytes and gives later fields their defaults (lbest_len NULL).
 * It must cover at least the fields through lbest (INVALID_ARG otherwise). */

int aco_construct_ex(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                     const int32_t *nnd, const float *eta_b, const void *grid, const float *tau,
                     int32_t m, int32_t ant0, double alpha, uint64_t seed, int64_t iteration,
                     const aco_construct_opts_t *opts, int32_t *tours, int64_t *lengths,
                     uint8_t *slots, float *step_prob, void *ws, size_t ws_bytes, void *stream);

/* Local bests (Algorithm 1): for every ant a with lengths[a] < lbest_len[a],
 * lbest[a] = tours[a] and lbest_len[a] = lengths[a] (strict improvement).
 * Initialise lbest_len to INT64_MAX to take the first tours.
 *   tours int32 [m][n], lengths int64 [m]; lbest int32 [m][n], lbest_len int64 [m]
 * Errors: INVALID_ARG. */
int aco_update_local_best(int32_t n, int32_t m, const int32_t *tours, const int64_t *lengths,
                          int32_t *lbest, int64_t *lbest_len, void *stream);

/* Pheromone from the ants' local best tours (the P-ACO variant of Section 3:
 * no evaporation; an edge of ant a's local best contributes the quality
 * ratio w_a = L_g / L_a in (0, 1], L_g the shortest local best):
 *     tau[i][r] = tau_base + delta * sum of w_a over the local bests that use
 *                 the edge {i, nn[i][r]}.
 * w_a is quantised as q_a = floor(2^shift * w_a) with the ratio in FP64 and
 * summed exactly in int64; tau = fl32(fl32(tau_base) + fl32(fl32(acc) *
 * fl32(delta * 2^-shift))), both directed slots of an edge equal.
 *   lbest int32 [m][n], lbest_len int64 [m] (> 0); tau float [n][k] (output)
 *   ws  aco_update_workspace_bytes(n, k, m) bytes
 * Every quantum is at most 2^shift and a slot sums at most m of them, so
 * m * 2^shift must stay below 2^63.
 * Errors: INVALID_ARG (sizes, shift outside [0, 62] or m * 2^shift >= 2^63,
 * tau_base or delta < 0 or not finite), WORKSPACE.  Device checks: a length
 * <= 0 (quantum 0), a tour entry out of range (edge skipped). */
int aco_pheromone_local_best(int32_t n, int32_t k, const int32_t *nn, const int8_t *rev,
                             int32_t m, const int32_t *lbest, const int64_t *lbest_len,
                             double tau_base, double delta, int32_t deposit_shift, float *tau,
                             void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Windowed 2-opt local search.  Section 4 applies 2-opt to a constructed
 * tour with a small probability (0.001); Section 5 limits it to pairs of
 * tour edges at most W = 500 positions apart.
 *
 * Tour a takes part when word 3 of the Philox block at counter
 * (0, a, iteration, 0) is below round(p 2^32) (words 0-2 are the start city
 * and PartialACO's plan).  Move (i, o), 2 <= o <= W' = min(W, n/2), j = i + o
 * (positions mod n), replaces the edges (t_i, t_i+1), (t_j, t_j+1) by
 * (t_i, t_j), (t_i+1, t_j+1), reversing t_i+1 .. t_j; its gain is
 *     g = d(t_i, t_j) + d(t_i+1, t_j+1) - d(t_i, t_i+1) - d(t_j, t_j+1).
 * Rounds: every position takes its best move (smallest g < 0, ties to the
 * smaller o); a move is applied when no move whose span (positions i..j+1)
 * meets its own is better by (g, i).  The applied moves are disjoint, their
 * gains add.  Rounds repeat until no move has g < 0 (the tour is 2-optimal
 * for all pairs of edges within W positions) or max_rounds rounds have
 * applied moves.
 * ------------------------------------------------------------------------ */

#define ACO_TWO_OPT_MAX_WINDOW 2048

typedef struct aco_two_opt_stats {
    int32_t selected;  /* tours that took part */
    int32_t converged; /* 1 when every such tour ended 2-optimal within the window */
    int64_t rounds;    /* rounds that applied moves (the largest over the tours) */
    int64_t moves;     /* moves applied, summed over the tours */
    int64_t gain;      /* their summed gains (<= 0): the change of the summed lengths */
} aco_two_opt_stats_t;

/* Workspace for m ants on n cities, handling up to `batch` tours at once. */
size_t aco_two_opt_workspace_bytes(int32_t n, int32_t m, int32_t batch);

/* Windowed 2-opt of the participating tours, in place.
 *   xy       int32 [n][2] coordinates
 *   tours    int32 [m][n] closed tours (permutations of 0..n-1), rewritten
 *   lengths  int64 [m] their lengths on entry; the gain is added
 *   slots    uint8 [m][n] or NULL: construction records; the positions whose
 *            incoming edge changed are set to 255 (no record), which the
 *            pheromone update then locates in the candidate lists
 *   window   W in [1, ACO_TWO_OPT_MAX_WINDOW] (W' < 2, i.e. n < 4 or W = 1,
 *            allows no move)
 *   p        participation probability in [0, 1]
 *   max_rounds  0: until no move improves; > 0: at most this many rounds
 *   stats    host pointer or NULL
 *   ws       aco_two_opt_workspace_bytes(n, m, batch) bytes, batch >= 1
 * Synchronises with `stream` once per call plus once per 16 rounds (the host
 * reads how many moves each round applied), and reports device checks (see
 * aco_device_error).
 * Errors: INVALID_ARG (sizes, window, p, NULL pointers), WORKSPACE, HIP, DEVICE. */
int aco_two_opt(const int32_t *xy, int32_t n, int32_t m, int32_t *tours, int64_t *lengths,
                uint8_t *slots, int32_t window, double p, uint64_t seed, int64_t iteration,
                int64_t max_rounds, int32_t batch, aco_two_opt_stats_t *stats, void *ws,
                size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Learned heuristic.  A small network scores every candidate edge from its
 * local geometry, and sigmoid(score) replaces eta = 1/d in the weights
 * tau^alpha * eta^beta of Eq. 1 (Section 2); the colony itself is unchanged.
 *
 * Features: FP32 [n][k][8] for candidate r of city i (j = nn[i][r], d_ir =
 * nnd[i][r], K = k - 1, or 1 when k = 1):
 *   0  d_ir / max(d_i0, 1)        1  d_ir / max(d_iK, 1)
 *   2  r / K                      3  rev[i][r] / K, or 1 if i is not in j's list
 *   4  cos, 5 sin of the angle from the edge i->j to c = sum over i's
 *      candidates s of (p_s - p_i) (cos 1, sin 0 when either vector is zero)
 *   6  d_iK / mean_c d_cK         7  d_jK / mean_c d_cK (both 1 if the mean is 0)
 * Each is an exactly rounded FP64 expression of integers, rounded once to FP32.
 *
 * Network (ACO_MLP_PARAMS FP32 parameters theta, row-major blocks at the
 * offsets below): W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [64], b3.
 * Weights W1, W2, W3 are rounded to BF16 (nearest-even) where they are used;
 * biases and accumulation are FP32; inputs are the features rounded to BF16:
 *   h1 = bf16(relu(W1 x + b1)), h2 = bf16(relu(W2 h1 + b2)), z = W3 . h2 + b3.
 * Training loss: mean over edges of w * BCE(sigmoid(z), y), w = pos_weight for
 * y = 1 and 1 for y = 0; labels y are 1 for candidate edges of a given tour.
 * ------------------------------------------------------------------------ */
#define ACO_MLP_PARAMS 4801
#define ACO_MLP_OFF_W1 0
#define ACO_MLP_OFF_B1 512
#define ACO_MLP_OFF_W2 576
#define ACO_MLP_OFF_B2 4672
#define ACO_MLP_OFF_W3 4736
#define ACO_MLP_OFF_B3 4800
#define ACO_MLP_OUT_LOGIT 0 /* out[e] = z */
#define ACO_MLP_OUT_ETA_B 1 /* out[e] = sigmoid(z)^beta (FP64, rounded once to FP32) */

/* Bytes of the workspace aco_edge_features needs (an exact integer sum). */
size_t aco_features_workspace_bytes(void);

/* The 8 features of every candidate edge.
 *   xy [n][2], nn/nnd [n][k], rev [n][k] as written by aco_build_candidates
 *   feat  float [n][k][8] (output, 16-byte aligned)
 * Errors: INVALID_ARG (n < 2, k out of [1, min(n-1, ACO_MAX_K)], NULL
 * pointer, misaligned feat), WORKSPACE. */
int aco_edge_features(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                      const int32_t *nnd, const int8_t *rev, float *feat, void *ws,
                      size_t ws_bytes, void *stream);

/* Forward pass over E edges (E = n*k when feat comes from aco_edge_features).
 *   feat  float [E][8] (16-byte aligned); theta float [ACO_MLP_PARAMS]
 *   out   float [E]: the logit (ACO_MLP_OUT_LOGIT) or, with ACO_MLP_OUT_ETA_B,
 *         the eta_b table that aco_construct_tours reads (sigmoid(z)^beta).
 * E = 0 does nothing.  Errors: INVALID_ARG. */
int aco_mlp_forward(const float *feat, int64_t E, const float *theta, int32_t mode,
                    double beta, float *out, void *stream);

/* Bytes of the workspace aco_mlp_backward needs for E edges. */
size_t aco_mlp_backward_workspace_bytes(int64_t E);

/* Gradient of the training loss over E >= 1 edges, with respect to theta
 * (weights through their BF16 values).  The gradients of the pre-activations
 * are rounded to BF16 where they enter the weight and input products, as the
 * matrix cores consume them.  Deterministic: partial sums are added in a
 * fixed order.
 *   labels uint8 [E] (0 or 1); pos_weight > 0
 *   grad  float [ACO_MLP_PARAMS] (output); loss double [1] (output, may be NULL)
 * Errors: INVALID_ARG, WORKSPACE. */
int aco_mlp_backward(const float *feat, const uint8_t *labels, int64_t E, const float *theta,
                     float pos_weight, float *grad, double *loss, void *ws, size_t ws_bytes,
                     void *stream);

/* One Adam step on the FP32 master parameters (in place), step >= 1:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   theta -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 *   theta, m, v, grad  float [ACO_MLP_PARAMS]   Errors: INVALID_ARG. */
int aco_mlp_adam(float *theta, float *m, float *v, const float *grad, int32_t step, float lr,
                 float beta1, float beta2, float eps, void *stream);

/* `steps` training steps in one call, t = first_step .. first_step+steps-1:
 * aco_mlp_backward on the batch of `batch` edges starting at edge
 * ((t - 1) mod floor(E / batch)) * batch, then aco_mlp_adam with step t.  The
 * result equals those calls made one by one (same kernels, same order).
 *   feat float [E][8], labels uint8 [E] (in the order the batches take them)
 *   theta, m, v float [ACO_MLP_PARAMS] (in/out); grad float [ACO_MLP_PARAMS]
 *   (scratch, holds the last gradient); loss: device double* (the last step's
 *   mean loss) or NULL
 *   ws  device workspace of aco_mlp_backward_workspace_bytes(batch) bytes
 * Errors: INVALID_ARG (1 <= batch <= E, first_step >= 1, steps >= 0, the
 * ranges of aco_mlp_backward and aco_mlp_adam), WORKSPACE. */
int aco_mlp_train(const float *feat, const uint8_t *labels, int64_t E, float *theta, float *m,
                  float *v, float pos_weight, int32_t first_step, int32_t steps, int64_t batch,
                  float lr, float beta1, float beta2, float eps, float *grad, double *loss,
                  void *ws, size_t ws_bytes, void *stream);

/* Training labels: labels[i][r] = 1 if {i, nn[i][r]} is an edge of the closed
 * tour (a permutation of 0..n-1), else 0.
 *   tour int32 [n]; labels uint8 [n][k] (output); pos_ws int32 [n] (scratch)
 * Errors: INVALID_ARG. */
int aco_tour_edge_labels(int32_t n, int32_t k, const int32_t *nn, const int32_t *tour,
                         uint8_t *labels, int32_t *pos_ws, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ACO_H */
