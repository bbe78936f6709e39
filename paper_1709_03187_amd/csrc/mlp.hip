// Learned edge heuristic: per-candidate-edge features, a BF16 MLP on the
// matrix cores (forward, and a fused forward+backward for training), Adam on
// FP32 master weights, and tour-edge labels.
//
// The score sigmoid(z) of the MLP stands in for eta = 1/d of the random
// proportional rule (Section 2, Eq. 1); everything else in the colony is
// unchanged.
//
// Matrix-core layout.  Activations are kept transposed (hidden unit x edge)
// so the output of one layer is the B operand of the next with no data
// movement.  For v_mfma_f32_16x16x16_bf16 on a 64-lane wave, with
// col = lane % 16 and grp = lane / 16:
//   A[i][k]: i = col, k = 4 grp + q   (4 BF16 per lane)
//   B[k][j]: k = 4 grp + q, j = col
//   D[i][j]: i = 4 grp + q, j = col   (4 FP32 per lane)
// A 16-edge tile puts edge j = col in every operand; a D block of hidden
// rows [16 b, 16 b + 16) is, after bias, ReLU and rounding, exactly the B
// operand of K-block b of the next layer.  Weight gradients contract over
// edges and need the transposed layout; those tiles go through LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aco.h"
#include "common.hpp"

namespace aco {
namespace {

constexpr int kF = 8, kH = 64;
constexpr int kOffW1 = 0, kOffB1 = 512, kOffW2 = 576, kOffB2 = 4672, kOffW3 = 4736, kOffB3 = 4800;
constexpr int kNParam = ACO_MLP_PARAMS;
static_assert(kOffB3 + 1 == kNParam, "parameter block layout");

constexpr int kWaves = 4;               // waves per workgroup of the MLP kernels
constexpr int kTile = 16;               // edges per wave per step
constexpr int kBackwardMaxBlocks = 256;   // one workgroup per CU at the kernel's occupancy

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest, ties to even (inputs here are finite): the
// hardware conversion (two values per instruction on gfx950).
__device__ inline short bf16_bits(float f) { return __builtin_bit_cast(short, (__bf16)f); }
__device__ inline float bf16_value(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }
__device__ inline float bf16_round(float f) { return bf16_value(bf16_bits(f)); }

__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ features
__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

// Sum over cities of the k-th candidate distance (exact, integer).
__global__ void k_sum_kth(const int32_t *nnd, int32_t n, int32_t k, unsigned long long *sum)
{
    __shared__ unsigned long long part[256 / 64];
    unsigned long long s = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        s += (unsigned long long)(uint32_t)nnd[i * k + (k - 1)];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
        atomicAdd(sum, t);
    }
}

// One thread per candidate slot (i, r).  Every value is formed with exactly
// rounded FP64 operations on integers and rounded once to FP32.
__global__ void k_features(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                           const int32_t *nnd, const int8_t *rev, const unsigned long long *kth_sum,
                           float *feat)
{
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * k) return;
    int64_t i = e / k;
    int r = (int)(e - i * k);
    const int32_t *row = nn + i * k;
    const int32_t *rowd = nnd + i * k;
    int32_t j = row[r];
    double km1 = k > 1 ? (double)(k - 1) : 1.0;
    double d = (double)rowd[r];
    double d0 = (double)max(rowd[0], 1);
    double dk = (double)max(rowd[k - 1], 1);
    float f[kF];
    f[0] = (float)__ddiv_rn(d, d0);
    f[1] = (float)__ddiv_rn(d, dk);
    f[2] = k > 1 ? (float)__ddiv_rn((double)r, km1) : 0.0f;
    int rv = rev[e];
    f[3] = rv >= 0 ? (float)__ddiv_rn((double)rv, km1) : 1.0f;

    int64_t xi = xy[2 * i], yi = xy[2 * i + 1];
    int64_t sx = 0, sy = 0;
    for (int s = 0; s < k; ++s) {
        int32_t c = row[s];
        sx += (int64_t)xy[2 * c] - xi;
        sy += (int64_t)xy[2 * c + 1] - yi;
    }
    double ex = (double)((int64_t)xy[2 * j] - xi), ey = (double)((int64_t)xy[2 * j + 1] - yi);
    double cx = (double)sx, cy = (double)sy;
    double dot = __dadd_rn(__dmul_rn(ex, cx), __dmul_rn(ey, cy));
    double crs = __dsub_rn(__dmul_rn(ex, cy), __dmul_rn(ey, cx));
    double ne = __dsqrt_rn(__dadd_rn(__dmul_rn(ex, ex), __dmul_rn(ey, ey)));
    double nc = __dsqrt_rn(__dadd_rn(__dmul_rn(cx, cx), __dmul_rn(cy, cy)));
    double den = __dmul_rn(ne, nc);
    if (den > 0.0) {
        f[4] = (float)__ddiv_rn(dot, den);
        f[5] = (float)__ddiv_rn(crs, den);
    } else {
        f[4] = 1.0f;
        f[5] = 0.0f;
    }
    double mean = __ddiv_rn((double)*kth_sum, (double)n);
    if (mean > 0.0) {
        f[6] = (float)__ddiv_rn((double)rowd[k - 1], mean);
        f[7] = (float)__ddiv_rn((double)nnd[(int64_t)j * k + (k - 1)], mean);
    } else {
        f[6] = 1.0f;
        f[7] = 1.0f;
    }
    float4 *out = reinterpret_cast<float4 *>(feat + e * kF);
    out[0] = make_float4(f[0], f[1], f[2], f[3]);
    out[1] = make_float4(f[4], f[5], f[6], f[7]);
}

// ------------------------------------------------------------------ network
// The weights one lane needs, as matrix-core operands (BF16) or FP32 values.
struct Net {
    bf16x4 w1[4];        // A of layer 1, block mb: W1[16 mb + col][4 grp + q] (0 for grp >= 2)
    bf16x4 w2[4][4];     // A of layer 2, block (mo, kb): W2[16 mo + col][16 kb + 4 grp + q]
    float w3[4][4];      // BF16 value of W3[16 m + 4 grp + q]
    float b1[4][4], b2[4][4], b3;
};

__device__ inline void load_net(const float *theta, int col, int grp, Net &N)
{
    for (int mb = 0; mb < 4; ++mb)
        for (int q = 0; q < 4; ++q) {
            N.w1[mb][q] = grp < 2 ? bf16_bits(theta[kOffW1 + (16 * mb + col) * kF + 4 * grp + q])
                                  : (short)0;
            int h = 16 * mb + 4 * grp + q;
            N.w3[mb][q] = bf16_round(theta[kOffW3 + h]);
            N.b1[mb][q] = theta[kOffB1 + h];
            N.b2[mb][q] = theta[kOffB2 + h];
            for (int kb = 0; kb < 4; ++kb)
                N.w2[mb][kb][q] = bf16_bits(theta[kOffW2 + (16 * mb + col) * kH + 16 * kb + 4 * grp + q]);
        }
    N.b3 = theta[kOffB3];
}

// B operand of layer 1 for edge e (features 4 grp .. 4 grp + 3; zero padding
// for grp >= 2 and for edges past the end).
__device__ inline bf16x4 load_x(const float *feat, int64_t e, bool valid, int grp)
{
    bf16x4 x = {0, 0, 0, 0};
    if (valid && grp < 2) {
        float4 v = *reinterpret_cast<const float4 *>(feat + e * kF + 4 * grp);
        x[0] = bf16_bits(v.x);
        x[1] = bf16_bits(v.y);
        x[2] = bf16_bits(v.z);
        x[3] = bf16_bits(v.w);
    }
    return x;
}

// Activations of one 16-edge tile, kept for the backward pass.
struct Acts {
    f32x4 a1[4], a2[4];  // pre-activations (D layout)
    bf16x4 h1[4];        // BF16 ReLU outputs of layer 1 (B layout of layer 2)
    float h2[4][4];      // BF16 values of the ReLU outputs of layer 2
};

// Forward pass of the tile; returns the logit of edge `col` (in every lane).
__device__ inline float forward_tile(const Net &N, bf16x4 x, Acts &A)
{
    for (int mb = 0; mb < 4; ++mb) {
        f32x4 c = {N.b1[mb][0], N.b1[mb][1], N.b1[mb][2], N.b1[mb][3]};
        c = mfma16(N.w1[mb], x, c);
        A.a1[mb] = c;
        for (int q = 0; q < 4; ++q) A.h1[mb][q] = bf16_bits(fmaxf(c[q], 0.0f));
    }
    for (int mo = 0; mo < 4; ++mo) {
        f32x4 c = {N.b2[mo][0], N.b2[mo][1], N.b2[mo][2], N.b2[mo][3]};
        for (int kb = 0; kb < 4; ++kb) c = mfma16(N.w2[mo][kb], A.h1[kb], c);
        A.a2[mo] = c;
        for (int q = 0; q < 4; ++q) A.h2[mo][q] = bf16_round(fmaxf(c[q], 0.0f));
    }
    float z = 0.0f;
    for (int mo = 0; mo < 4; ++mo)
        for (int q = 0; q < 4; ++q) z += N.w3[mo][q] * A.h2[mo][q];
    z += __shfl_xor(z, 16);
    z += __shfl_xor(z, 32);
    return z + N.b3;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *feat, int64_t E,
                                                     const float *theta, int mode, double beta,
                                                     float *out)
{
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
    Net N;
    load_net(theta, col, grp, N);
    int64_t nw = (int64_t)gridDim.x * kWaves;
    int64_t t = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    // the next tile's features are loaded while this tile is computed
    bf16x4 xn = load_x(feat, t * kTile + col, t * kTile + col < E, grp);
    // every lane ends a tile with the logit of edge `col`; the output of
    // tile number u goes out from the lanes of group u mod 4, so the FP64
    // sigmoid and power run once per four tiles on all 64 lanes
    float zk = 0.0f;
    int64_t ek = -1;   // edge whose output this lane holds, or -1
    int slot = 0;
    for (; t * kTile < E; t += nw) {
        int64_t e = t * kTile + col;
        bool valid = e < E;
        const bf16x4 x = xn;
        const int64_t en = (t + nw) * kTile + col;
        xn = load_x(feat, en, en < E, grp);
        Acts A;
        float z = forward_tile(N, x, A);
        if (grp == slot) {
            zk = z;
            ek = valid ? e : -1;
        }
        if (++slot == 4 || (t + nw) * kTile >= E) {   // wave-uniform
            if (ek >= 0) {
                if (mode == ACO_MLP_OUT_LOGIT) {
                    out[ek] = zk;
                } else {
                    double sg = 1.0 / (1.0 + exp(-(double)zk));
                    out[ek] = (float)pow(sg, beta);
                }
            }
            ek = -1;
            slot = 0;
        }
    }
}

// Per-wave LDS staging for the transposes of one tile (BF16 bits).
struct Stage {
    short d2[kH * kTile];   // [hidden][edge]
    short h1[kH * kTile];
    short d1[kH * kTile];
    short x[kTile * kF];    // [edge][feature]
};
// LDS of the backward kernel: the waves' staging areas while tiles run, then
// one row of gradient sums per wave (and a loss sum per wave) for the
// workgroup's reduction
constexpr size_t kGradRowBytes = (sizeof(float) * kNParam + 15) & ~(size_t)15;
constexpr size_t kStageBytes = sizeof(Stage) * kWaves;
constexpr size_t kReduceBytes = kGradRowBytes * kWaves + sizeof(double) * kWaves;
constexpr size_t kBackwardLds = kStageBytes > kReduceBytes ? kStageBytes : kReduceBytes;

__device__ inline float sum16(float v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}
__device__ inline double sum16d(double v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// Fused forward + backward of the weighted mean BCE over edges [0, E).
// Each workgroup writes its partial gradient (and loss sum) to its own row of
// `partial`; the reduction kernel adds the rows in a fixed order, so the
// result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_mlp_backward(const float *feat, const uint8_t *labels,
                                                      int64_t E, const float *theta,
                                                      float pos_weight, float inv_e,
                                                      float *partial, double *loss_partial)
{
    extern __shared__ __align__(16) unsigned char lds[];   // kBackwardLds bytes
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
    Stage &S = reinterpret_cast<Stage *>(lds)[wave];
    Net N;
    load_net(theta, col, grp, N);
    // A of the data gradient d1 = W2^T d2: block (mi, ko) holds W2[16 ko + 4 grp + q][16 mi + col]
    bf16x4 w2t[4][4];
    for (int mi = 0; mi < 4; ++mi)
        for (int ko = 0; ko < 4; ++ko)
            for (int q = 0; q < 4; ++q)
                w2t[mi][ko][q] =
                    bf16_bits(theta[kOffW2 + (16 * ko + 4 * grp + q) * kH + 16 * mi + col]);

    f32x4 gw2[4][4], gw1[4];
    float gw3[4][4], gb2[4][4], gb1[4][4], gb3 = 0.0f;
    double lsum = 0.0;
    for (int a = 0; a < 4; ++a) {
        gw1[a] = f32x4{0, 0, 0, 0};
        for (int b = 0; b < 4; ++b) {
            gw2[a][b] = f32x4{0, 0, 0, 0};
            gw3[a][b] = gb2[a][b] = gb1[a][b] = 0.0f;
        }
    }

    // the loop bound is uniform over the workgroup (a barrier follows the loop)
    for (int64_t base = (int64_t)blockIdx.x * kWaves; base * kTile < E;
         base += (int64_t)gridDim.x * kWaves) {
        int64_t e = (base + wave) * kTile + col;
        bool valid = e < E;
        bf16x4 x = load_x(feat, e, valid, grp);
        Acts A;
        float z = forward_tile(N, x, A);
        float y = valid ? (float)labels[e] : 0.0f;
        float w = y > 0.5f ? pos_weight : 1.0f;
        float s = 1.0f / (1.0f + expf(-z));
        float g = valid ? w * (s - y) * inv_e : 0.0f;
        if (grp == 0 && valid) {
            float sp = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
            lsum += (double)(w * (sp - y * z));
            gb3 += g;
        }
        // output layer and the gradient at a2
        bf16x4 d2b[4];
        for (int mo = 0; mo < 4; ++mo)
            for (int q = 0; q < 4; ++q) {
                gw3[mo][q] += g * A.h2[mo][q];
                float d2 = A.a2[mo][q] > 0.0f ? N.w3[mo][q] * g : 0.0f;
                gb2[mo][q] += d2;
                d2b[mo][q] = bf16_bits(d2);
            }
        // gradient at a1: D[in][e] = sum_out W2[out][in] d2[out][e]
        bf16x4 d1b[4];
        for (int mi = 0; mi < 4; ++mi) {
            f32x4 c = {0, 0, 0, 0};
            for (int ko = 0; ko < 4; ++ko) c = mfma16(w2t[mi][ko], d2b[ko], c);
            for (int q = 0; q < 4; ++q) {
                float d1 = A.a1[mi][q] > 0.0f ? c[q] : 0.0f;
                gb1[mi][q] += d1;
                d1b[mi][q] = bf16_bits(d1);
            }
        }
        // stage [hidden][edge] tiles for the edge-contracting products
        for (int m = 0; m < 4; ++m)
            for (int q = 0; q < 4; ++q) {
                int at = (16 * m + 4 * grp + q) * kTile + col;
                S.d2[at] = d2b[m][q];
                S.h1[at] = A.h1[m][q];
                S.d1[at] = d1b[m][q];
            }
        if (grp < 2)
            for (int q = 0; q < 4; ++q) S.x[col * kF + 4 * grp + q] = x[q];
        // the staging area is this wave's own: its LDS operations complete in
        // order, so only the compiler's ordering needs pinning
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // dW2[out][in] += sum_e d2[out][e] h1[in][e]; dW1[h][f] += sum_e d1[h][e] x[e][f]
        bf16x4 ad2[4], bh1[4];
        for (int m = 0; m < 4; ++m) {
            ad2[m] = *reinterpret_cast<const bf16x4 *>(&S.d2[(16 * m + col) * kTile + 4 * grp]);
            bh1[m] = *reinterpret_cast<const bf16x4 *>(&S.h1[(16 * m + col) * kTile + 4 * grp]);
        }
        bf16x4 bx;
        for (int q = 0; q < 4; ++q) bx[q] = col < kF ? S.x[(4 * grp + q) * kF + col] : (short)0;
        for (int mh = 0; mh < 4; ++mh) {
            bf16x4 ad1 = *reinterpret_cast<const bf16x4 *>(&S.d1[(16 * mh + col) * kTile + 4 * grp]);
            gw1[mh] = mfma16(ad1, bx, gw1[mh]);
        }
        for (int mo = 0; mo < 4; ++mo)
            for (int mi = 0; mi < 4; ++mi) gw2[mo][mi] = mfma16(ad2[mo], bh1[mi], gw2[mo][mi]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();   // every wave is done with its staging area

    // sums over the 16 edge columns held by the lanes of a row
    for (int a = 0; a < 4; ++a)
        for (int q = 0; q < 4; ++q) {
            gw3[a][q] = sum16(gw3[a][q]);
            gb2[a][q] = sum16(gb2[a][q]);
            gb1[a][q] = sum16(gb1[a][q]);
        }
    gb3 = sum16(gb3);
    lsum = sum16d(lsum);

    // each wave writes its whole gradient row (every parameter is held by
    // exactly one lane of a wave), then the rows are added in wave order
    float *red = reinterpret_cast<float *>(lds + (size_t)wave * kGradRowBytes);
    double *lred = reinterpret_cast<double *>(lds + (size_t)kWaves * kGradRowBytes);
    for (int mo = 0; mo < 4; ++mo)
        for (int mi = 0; mi < 4; ++mi)
            for (int q = 0; q < 4; ++q)
                red[kOffW2 + (16 * mo + 4 * grp + q) * kH + 16 * mi + col] = gw2[mo][mi][q];
    if (col < kF)
        for (int mh = 0; mh < 4; ++mh)
            for (int q = 0; q < 4; ++q) red[kOffW1 + (16 * mh + 4 * grp + q) * kF + col] = gw1[mh][q];
    if (col == 0)
        for (int m = 0; m < 4; ++m)
            for (int q = 0; q < 4; ++q) {
                int h = 16 * m + 4 * grp + q;
                red[kOffW3 + h] = gw3[m][q];
                red[kOffB2 + h] = gb2[m][q];
                red[kOffB1 + h] = gb1[m][q];
            }
    if (lane == 0) {
        red[kOffB3] = gb3;
        lred[wave] = lsum;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < kNParam; p += blockDim.x) {
        float t = reinterpret_cast<const float *>(lds)[p];
        for (int wv = 1; wv < kWaves; ++wv)
            t += reinterpret_cast<const float *>(lds + (size_t)wv * kGradRowBytes)[p];
        partial[(int64_t)blockIdx.x * kNParam + p] = t;
    }
    if (threadIdx.x == 0) {
        double t = lred[0];
        for (int wv = 1; wv < kWaves; ++wv) t += lred[wv];
        loss_partial[blockIdx.x] = t;
    }
}

// Sum of the workgroups' partial rows, 64 parameters per block of 16 waves:
// wave q adds rows q, q + 16, q + 32, ... (at most 16 rows for the largest
// grid, all loads independent, four interleaved accumulators); the 16 wave
// sums are then added in order q = 0..15.  The loss partials are added by the
// first wave of block 0: lane l adds rows l, l + 64, ... in order, then a
// fixed butterfly.  The order depends only on the number of rows, so results
// are reproducible.
constexpr int kReduceWaves = 16;
__global__ __launch_bounds__(64 * kReduceWaves) void k_mlp_reduce(const float *partial,
                                                                  const double *loss_partial,
                                                                  int blocks, double inv_e,
                                                                  float *grad, double *loss)
{
    __shared__ float part[kReduceWaves][64];
    const int pl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + pl;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    if (p < kNParam) {
        constexpr int S = kReduceWaves;
        int b = q;
        for (; b + 3 * S < blocks; b += 4 * S) {
            a0 += partial[(int64_t)b * kNParam + p];
            a1 += partial[(int64_t)(b + S) * kNParam + p];
            a2 += partial[(int64_t)(b + 2 * S) * kNParam + p];
            a3 += partial[(int64_t)(b + 3 * S) * kNParam + p];
        }
        for (; b < blocks; b += S) a0 += partial[(int64_t)b * kNParam + p];
    }
    part[q][pl] = (a0 + a1) + (a2 + a3);
    if (blockIdx.x == 0 && q == 0 && loss) {
        double t = 0.0;
        for (int b = pl; b < blocks; b += 64) t += loss_partial[b];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
        if (pl == 0) *loss = t * inv_e;
    }
    __syncthreads();
    if (q == 0 && p < kNParam) {
        float t = part[0][pl];
        for (int w = 1; w < kReduceWaves; ++w) t += part[w][pl];
        grad[p] = t;
    }
}

__global__ void k_adam(float *theta, float *m, float *v, const float *grad, int count, float lr,
                       float beta1, float beta2, float eps, float c1, float c2)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    float g = grad[p];
    float mp = beta1 * m[p] + (1.0f - beta1) * g;
    float vp = beta2 * v[p] + (1.0f - beta2) * (g * g);
    m[p] = mp;
    v[p] = vp;
    float mh = mp / c1, vh = vp / c2;
    theta[p] = theta[p] - lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_tour_positions(const int32_t *tour, int32_t n, int32_t *pos)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int32_t c = tour[t];
    if (c >= 0 && c < n) pos[c] = t;
}

__global__ void k_edge_labels(int32_t n, int32_t k, const int32_t *nn, const int32_t *pos,
                              uint8_t *labels)
{
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * k) return;
    int64_t i = e / k;
    int32_t j = nn[e];
    if (j < 0 || j >= n) {
        labels[e] = 0;
        return;
    }
    int32_t d = pos[i] - pos[j];
    labels[e] = (d == 1 || d == -1 || d == n - 1 || d == 1 - n) ? 1 : 0;
}

int backward_blocks(int64_t E)
{
    int64_t per = (int64_t)kWaves * kTile;
    int64_t b = (E + per - 1) / per;
    return (int)(b < 1 ? 1 : (b > kBackwardMaxBlocks ? kBackwardMaxBlocks : b));
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace aco

using namespace aco;

extern "C" size_t aco_features_workspace_bytes(void) { return 256; }

extern "C" int aco_edge_features(const int32_t *xy, int32_t n, int32_t k, const int32_t *nn,
                                 const int32_t *nnd, const int8_t *rev, float *feat, void *ws,
                                 size_t ws_bytes, void *stream)
{
    clear_error();
    ACO_REQUIRE(n >= 2 && n <= (1 << 27), "n = %d out of range [2, 2^27]", n);
    ACO_REQUIRE(k >= 1 && k <= ACO_MAX_K && k <= n - 1, "k = %d out of range [1, min(n-1, %d)]", k,
                ACO_MAX_K);
    ACO_REQUIRE(xy && nn && nnd && rev && feat, "a required pointer is NULL");
    ACO_REQUIRE(((uintptr_t)feat & 15) == 0, "feat must be 16-byte aligned");
    if (!ws || ws_bytes < aco_features_workspace_bytes())
        return fail(ACO_ERR_WORKSPACE, "workspace of %zu bytes is smaller than %zu", ws_bytes,
                    aco_features_workspace_bytes());
    hipStream_t st = as_stream(stream);
    auto *sum = reinterpret_cast<unsigned long long *>(ws);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, sum);
    ACO_LAUNCH_CHECK("k_zero_u64");
    unsigned sb = blocks_for(n, 256);
    hipLaunchKernelGGL(k_sum_kth, dim3(sb > 1024 ? 1024 : sb), dim3(256), 0, st, nnd, n, k, sum);
    ACO_LAUNCH_CHECK("k_sum_kth");
    hipLaunchKernelGGL(k_features, dim3(blocks_for((int64_t)n * k, 256)), dim3(256), 0, st, xy, n,
                       k, nn, nnd, rev, sum, feat);
    ACO_LAUNCH_CHECK("k_features");
    return ACO_OK;
}

static int check_mlp_args(const float *feat, int64_t E, const float *theta)
{
    ACO_REQUIRE(E >= 0 && E <= ((int64_t)1 << 40), "E = %lld out of range", (long long)E);
    ACO_REQUIRE(theta, "theta is NULL");
    ACO_REQUIRE(E == 0 || feat, "feat is NULL");
    ACO_REQUIRE(((uintptr_t)feat & 15) == 0, "feat must be 16-byte aligned");
    return ACO_OK;
}

static unsigned forward_blocks(int64_t E)
{
    int64_t per = (int64_t)kWaves * kTile;
    int64_t b = (E + per - 1) / per;
    // one round of resident waves (three per SIMD at the kernel's registers):
    // each wave loads the network once and runs many tiles
    const int64_t cap = (int64_t)3 * num_cus();
    return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

extern "C" int aco_mlp_forward(const float *feat, int64_t E, const float *theta, int32_t mode,
                               double beta, float *out, void *stream)
{
    clear_error();
    int rc = check_mlp_args(feat, E, theta);
    if (rc) return rc;
    ACO_REQUIRE(mode == ACO_MLP_OUT_LOGIT || mode == ACO_MLP_OUT_ETA_B, "mode = %d unknown", mode);
    ACO_REQUIRE(beta >= 0.0 && beta <= 1e6, "beta = %g out of range", beta);
    ACO_REQUIRE(E == 0 || out, "out is NULL");
    if (E == 0) return ACO_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3(forward_blocks(E)), dim3(64 * kWaves), 0,
                       as_stream(stream), feat, E, theta, (int)mode, beta, out);
    ACO_LAUNCH_CHECK("k_mlp_forward");
    return ACO_OK;
}

extern "C" size_t aco_mlp_backward_workspace_bytes(int64_t E)
{
    if (E < 0) return 0;
    size_t G = (size_t)backward_blocks(E);
    return align256(G * kNParam * sizeof(float)) + align256(G * sizeof(double));
}

extern "C" int aco_mlp_backward(const float *feat, const uint8_t *labels, int64_t E,
                                const float *theta, float pos_weight, float *grad, double *loss,
                                void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_mlp_args(feat, E, theta);
    if (rc) return rc;
    ACO_REQUIRE(E >= 1, "E must be >= 1 (the loss is a mean over edges)");
    ACO_REQUIRE(labels && grad, "a required pointer is NULL");
    ACO_REQUIRE(pos_weight > 0.0f && pos_weight < 1e6f, "pos_weight = %g out of range",
                (double)pos_weight);
    size_t need = aco_mlp_backward_workspace_bytes(E);
    if (!ws || ws_bytes < need)
        return fail(ACO_ERR_WORKSPACE, "workspace of %zu bytes is smaller than %zu", ws_bytes, need);
    int G = backward_blocks(E);
    auto *partial = reinterpret_cast<float *>(ws);
    auto *lpart = reinterpret_cast<double *>(static_cast<char *>(ws) +
                                             align256((size_t)G * kNParam * sizeof(float)));
    hipStream_t st = as_stream(stream);
    if (kBackwardLds > 65536)
        ACO_HIP_CHECK(hipFuncSetAttribute((const void *)k_mlp_backward,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)kBackwardLds));
    hipLaunchKernelGGL(k_mlp_backward, dim3(G), dim3(64 * kWaves), kBackwardLds, st, feat, labels,
                       E, theta, pos_weight, (float)(1.0 / (double)E), partial, lpart);
    ACO_LAUNCH_CHECK("k_mlp_backward");
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParam + 63) / 64), dim3(64 * kReduceWaves), 0, st,
                       partial, lpart, G, 1.0 / (double)E, grad, loss);
    ACO_LAUNCH_CHECK("k_mlp_reduce");
    return ACO_OK;
}

extern "C" int aco_mlp_adam(float *theta, float *m, float *v, const float *grad, int32_t step,
                            float lr, float beta1, float beta2, float eps, void *stream)
{
    clear_error();
    ACO_REQUIRE(theta && m && v && grad, "a required pointer is NULL");
    ACO_REQUIRE(step >= 1, "step = %d must be >= 1", step);
    ACO_REQUIRE(lr >= 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f &&
                    eps > 0.0f,
                "Adam hyper-parameters out of range");
    float c1 = (float)(1.0 - pow((double)beta1, (double)step));
    float c2 = (float)(1.0 - pow((double)beta2, (double)step));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(kNParam, 256)), dim3(256), 0, as_stream(stream),
                       theta, m, v, grad, kNParam, lr, beta1, beta2, eps, c1, c2);
    ACO_LAUNCH_CHECK("k_adam");
    return ACO_OK;
}

// Several training steps in one call: the same kernels as aco_mlp_backward
// followed by aco_mlp_adam, step after step, with no host round trip between
// them (the per-step host work of a caller loop is what bounds training).
extern "C" int aco_mlp_train(const float *feat, const uint8_t *labels, int64_t E, float *theta,
                             float *m, float *v, float pos_weight, int32_t first_step,
                             int32_t steps, int64_t batch, float lr, float beta1, float beta2,
                             float eps, float *grad, double *loss, void *ws, size_t ws_bytes,
                             void *stream)
{
    clear_error();
    int rc = check_mlp_args(feat, E, theta);
    if (rc) return rc;
    ACO_REQUIRE(labels && m && v && grad, "a required pointer is NULL");
    ACO_REQUIRE(first_step >= 1 && steps >= 0 && (int64_t)first_step + steps - 1 <= INT32_MAX,
                "steps %d.. (%d of them) out of range", first_step, steps);
    ACO_REQUIRE(batch >= 1 && batch <= E, "batch = %lld out of [1, E]", (long long)batch);
    ACO_REQUIRE(pos_weight > 0.0f && pos_weight < 1e6f, "pos_weight = %g out of range",
                (double)pos_weight);
    ACO_REQUIRE(lr >= 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f &&
                    eps > 0.0f,
                "Adam hyper-parameters out of range");
    const size_t need = aco_mlp_backward_workspace_bytes(batch);
    if (!ws || ws_bytes < need)
        return fail(ACO_ERR_WORKSPACE, "workspace of %zu bytes is smaller than %zu", ws_bytes, need);
    const int64_t chunks = E / batch;   // >= 1
    for (int32_t s = 0; s < steps; ++s) {
        const int32_t t = first_step + s;
        const int64_t lo = ((int64_t)(t - 1) % chunks) * batch;
        rc = aco_mlp_backward(feat + lo * kF, labels + lo, batch, theta, pos_weight, grad,
                              s + 1 == steps ? loss : nullptr, ws, ws_bytes, stream);
        if (rc) return rc;
        rc = aco_mlp_adam(theta, m, v, grad, t, lr, beta1, beta2, eps, stream);
        if (rc) return rc;
    }
    return ACO_OK;
}

extern "C" int aco_tour_edge_labels(int32_t n, int32_t k, const int32_t *nn, const int32_t *tour,
                                    uint8_t *labels, int32_t *pos_ws, void *stream)
{
    clear_error();
    ACO_REQUIRE(n >= 3 && n <= (1 << 27), "n = %d out of range [3, 2^27]", n);
    ACO_REQUIRE(k >= 1 && k <= ACO_MAX_K && k <= n - 1, "k = %d out of range", k);
    ACO_REQUIRE(nn && tour && labels && pos_ws, "a required pointer is NULL");
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_tour_positions, dim3(blocks_for(n, 256)), dim3(256), 0, st, tour, n,
                       pos_ws);
    ACO_LAUNCH_CHECK("k_tour_positions");
    hipLaunchKernelGGL(k_edge_labels, dim3(blocks_for((int64_t)n * k, 256)), dim3(256), 0, st, n,
                       k, nn, pos_ws, labels);
    ACO_LAUNCH_CHECK("k_edge_labels");
    return ACO_OK;
}
