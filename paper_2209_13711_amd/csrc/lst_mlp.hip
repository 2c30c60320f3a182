// Learned scorer of triplets and quintuplets: MLP 40 -> 64 -> 64 -> 1
// (ReLU, ReLU, logit), one network per object kind.
//
// Inference runs on the gfx950 matrix cores.  A wavefront takes 16
// candidates at a time; layers 1 and 2 are v_mfma_f32_16x16x32_bf16
// products (BF16 operands, FP32 accumulation), the first hidden layer is
// rounded to BF16 (nearest, ties to even) before it feeds the second, and
// the last layer is an FP32 dot product on the vector ALUs (N = 1 would
// waste a matrix tile).  In the chain the 40 features of a quintuplet are
// computed in registers by the lane that owns it, standardised and written
// straight into the LDS operand tile, so they never travel through HBM.
//
// Training uses the same forward tile (saving the hidden activations), a
// backward pass in FP32 with one thread per row for the row-local terms and
// one thread per parameter and row chunk for the batch sums, followed by a
// reduction over the chunks in a fixed order (gradients are bit-for-bit
// deterministic), and Adam on FP32 master weights.
//
// Parameter vector (FP32): W1[64][40] (row = hidden unit), b1[64],
// W2[64][64], b2[64], w3[64], b3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "lst_access.hpp"
#include "lst_cuts.hpp"

namespace lst {

constexpr int NIN = MLP_NIN, NH = MLP_NH, KP = 64;  // inputs, hidden units, padded K
constexpr int LD = KP + 8;   // LDS row stride in BF16 elements (144 B: conflict-free b128 reads)
constexpr int OFF_W1 = 0, OFF_B1 = NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == MLP_NPARAM, "parameter layout");
constexpr int GRAD_CHUNKS = 64;   // row chunks of the gradient sums

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> BF16 bits, round to nearest even (a NaN stays a quiet NaN)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// eight consecutive BF16 values (16 bytes, 16-byte aligned) as an MFMA operand
__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

// Weights in LDS as BF16 [output unit][k] (K zero padded), the rest FP32.
struct MlpW {
    uint16_t w1[NH][LD];
    uint16_t w2[NH][LD];
    float b1[NH], b2[NH], w3[NH];
    float b3;
};

// Every kernel that stages the weights runs BLOCK threads: each thread loads
// its WPT elements of each matrix before it converts them, so the loads are
// in flight together rather than one after the other.
constexpr int WPT = NH * KP / BLOCK;
static_assert(NH * KP % BLOCK == 0 && NH * NH == NH * KP, "weight staging");

__device__ __forceinline__ void load_weights(const float *P, MlpW &w)
{
    float a[WPT], b[WPT];
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
        const int i = threadIdx.x + u * BLOCK, o = i / KP, k = i % KP;
        a[u] = k < NIN ? P[OFF_W1 + o * NIN + k] : 0.0f;
        b[u] = P[OFF_W2 + o * NH + k];
    }
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
        const int i = threadIdx.x + u * BLOCK, o = i / KP, k = i % KP;
        w.w1[o][k] = k < NIN ? f2bf(a[u]) : (uint16_t)0;
        w.w2[o][k] = f2bf(b[u]);
    }
    for (int i = threadIdx.x; i < NH; i += blockDim.x) {
        w.b1[i] = P[OFF_B1 + i];
        w.b2[i] = P[OFF_B2 + i];
        w.w3[i] = P[OFF_W3 + i];
    }
    if (threadIdx.x == 0) w.b3 = P[OFF_B3];
}

// orders a wave's LDS writes before later LDS reads by other lanes of the
// same wave (a wave's LDS operations complete in issue order): the operand
// and hidden tiles are wave-private, so no block barrier is needed for them
__device__ __forceinline__ void wave_tile_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc[nt] = A(16 x 64) * W(rows 16 nt .. 16 nt + 15)^T.  Operand layouts of
// v_mfma_f32_16x16x32_bf16 on a wave64: lane l supplies row l%16 of A and
// column l%16 of B, each with the eight k values 8 (l/16) .. +7 of the
// 32-wide k step; lane l receives D rows 4 (l/16) + r, column l%16.
__device__ __forceinline__ void mfma_layer(const uint16_t (*A)[LD], const uint16_t (*W)[LD],
                                           f32x4 acc[4])
{
    const int l = threadIdx.x & 63;
    const int row = l & 15, kq = 8 * (l >> 4);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < KP / 32; ++ks) {
        const bf16x8 a = load8(&A[row][32 * ks + kq]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x8 b = load8(&W[16 * nt + row][32 * ks + kq]);
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nt], 0, 0, 0);
        }
    }
}

// Forward of the 16 rows in A (wave-private), H a wave-private 16-row
// scratch tile.  Lanes with l%16 == 0 return the logits of rows
// 4 (l/16) + r in logit[r].  If h1_out / h2_out are given, rows row0 + i < n
// of the first (BF16, stride KP) and second (FP32, stride NH) hidden layers
// are stored.  A and H are the calling wave's own tiles.
__device__ __forceinline__ void mlp_tile(const MlpW &w, const uint16_t (*A)[LD], uint16_t (*H)[LD],
                                         float logit[4], uint16_t *h1_out, float *h2_out,
                                         int64_t row0, int64_t n)
{
    const int l = threadIdx.x & 63;
    const int col = l & 15, rq = 4 * (l >> 4);
    f32x4 acc[4];
    mfma_layer(A, w.w1, acc);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = 16 * nt + col;
            const float z = acc[nt][r] + w.b1[j];
            const uint16_t hb = f2bf(z > 0.0f ? z : 0.0f);
            H[rq + r][j] = hb;
            if (h1_out && row0 + rq + r < n) h1_out[(row0 + rq + r) * KP + j] = hb;
        }
    wave_tile_sync();
    mfma_layer(H, w.w2, acc);
    float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = 16 * nt + col;
            const float z = acc[nt][r] + w.b2[j];
            const float h2 = z > 0.0f ? z : 0.0f;
            if (h2_out && row0 + rq + r < n) h2_out[(row0 + rq + r) * NH + j] = h2;
            part[r] += h2 * w.w3[j];
        }
    // sum over the 16 lanes that hold one row's hidden units
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float v = part[r];
        v += __shfl_xor(v, 8, 16);
        v += __shfl_xor(v, 4, 16);
        v += __shfl_xor(v, 2, 16);
        v += __shfl_xor(v, 1, 16);
        logit[r] = v + w.b3;
    }
    wave_tile_sync();   // H is reused by the next tile
}

// ---------------------------------------------------------------- training forward
struct SmFwd {
    MlpW w;
    uint16_t x[WAVES][16][LD];
    uint16_t h[WAVES][16][LD];
};

// X: [n][KP] BF16 rows (features standardised, zero padded).
__global__ __launch_bounds__(BLOCK) void k_mlp_forward(const float *P, const uint16_t *X, int64_t n,
                                                       float *logits, uint16_t *h1, float *h2)
{
    __shared__ SmFwd sm;
    load_weights(P, sm.w);
    __syncthreads();   // weights staged
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t tiles = (n + 15) / 16;
    for (int64_t base = (int64_t)blockIdx.x * WAVES; base < tiles; base += (int64_t)gridDim.x * WAVES) {
        const int64_t tile = base + w;
        const int64_t row0 = tile * 16;
        const bool live = tile < tiles;
        // stage the tile, 16 bytes per lane and step (rows beyond n are zero)
        for (int i = l; i < 16 * (KP / 8); i += 64) {
            const int r = i / (KP / 8), c8 = (i % (KP / 8)) * 8;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (live && row0 + r < n) v = *reinterpret_cast<const uint4 *>(&X[(row0 + r) * KP + c8]);
            *reinterpret_cast<uint4 *>(&sm.x[w][r][c8]) = v;
        }
        wave_tile_sync();
        float lg[4];
        mlp_tile(sm.w, sm.x[w], sm.h[w], lg, live ? h1 : nullptr, live ? h2 : nullptr, row0, n);
        if ((l & 15) == 0 && live)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gr = row0 + 4 * (l >> 4) + r;
                if (gr < n) logits[gr] = lg[r];
            }
    }
}

// standardise raw FP32 features [n][40] into BF16 rows of KP (zero padded)
__global__ void k_mlp_prepare(const float *F, const float *mean, const float *istd, int64_t n,
                              uint16_t *X)
{
    const int64_t tot = n * KP;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / KP;
        const int k = (int)(i % KP);
        X[i] = k < NIN ? f2bf((F[r * NIN + k] - mean[k]) * istd[k]) : (uint16_t)0;
    }
}

// ---------------------------------------------------------------- training backward
// Row-local terms of the gradient of the mean BCE-with-logits loss:
// g = (sigmoid(z) - y) / n, dz2 = g w3 [h2 > 0], dz1 = (dz2 W2) [h1 > 0],
// with W2 the BF16-rounded weights the forward used; also the per-row loss.
// A block takes ROWS_PER_BLOCK rows, ROW_GROUPS at a time: 64 lanes per row,
// lane j writes dz2[r][j] and lane k sums dz1[r][k] over j = 0..63 in order,
// so every output is coalesced and the sums run in a fixed order.
constexpr int ROW_GROUPS = BLOCK / NH, ROWS_PER_BLOCK = 2 * ROW_GROUPS;

__global__ __launch_bounds__(BLOCK) void k_mlp_rows(const float *P, const float *logits,
                                                    const uint8_t *y, int64_t n, const uint16_t *h1,
                                                    const float *h2, float *g, float *dz2,
                                                    float *dz1, float *loss_rows)
{
    __shared__ float w2[NH][NH + 1];
    __shared__ float w3[NH];
    __shared__ float d2[ROW_GROUPS][NH];
    {
        float b[WPT];   // all loads in flight, then the BF16 rounding
#pragma unroll
        for (int u = 0; u < WPT; ++u) b[u] = P[OFF_W2 + threadIdx.x + u * BLOCK];
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int i = threadIdx.x + u * BLOCK;
            w2[i / NH][i % NH] = bf2f(f2bf(b[u]));
        }
    }
    for (int i = threadIdx.x; i < NH; i += blockDim.x) w3[i] = P[OFF_W3 + i];
    const int grp = threadIdx.x / NH, lane = threadIdx.x % NH;
    for (int64_t b = (int64_t)blockIdx.x * ROWS_PER_BLOCK; b < n;
         b += (int64_t)gridDim.x * ROWS_PER_BLOCK) {
        __syncthreads();                     // weights loaded; d2 of the last rows consumed
        for (int q = 0; q < ROWS_PER_BLOCK; q += ROW_GROUPS) {
            const int64_t r = b + q + grp;
            if (r < n) {
                const float z = logits[r];
                const float yv = y[r] ? 1.0f : 0.0f;
                const float gr = (1.0f / (1.0f + expf(-z)) - yv) / (float)n;
                if (lane == 0) {
                    loss_rows[r] = (z > 0.0f ? z : 0.0f) - z * yv + log1pf(expf(-fabsf(z)));
                    g[r] = gr;
                }
                const float dj = h2[r * NH + lane] > 0.0f ? gr * w3[lane] : 0.0f;
                d2[grp][lane] = dj;
                dz2[r * NH + lane] = dj;
            }
            __syncthreads();
            if (r < n) {
                float acc = 0.0f;
#pragma unroll
                for (int j = 0; j < NH; ++j) acc += d2[grp][j] * w2[j][lane];
                dz1[r * NH + lane] = h1[r * KP + lane] != 0 ? acc : 0.0f;
            }
            __syncthreads();                 // d2 is rewritten by the next rows
        }
    }
}

// Sums over the rows r0..r1-1 in row order of a(r) b(r) (or of a(r)):
// GP_U rows' operands are loaded before they are added, so GP_U loads are in
// flight at once; the additions keep the row order.
constexpr int GP_U = 16;

template <class A, class B>
__device__ __forceinline__ float rows_dot(int64_t r0, int64_t r1, A a, B b)
{
    float acc = 0.0f;
    for (int64_t rb = r0; rb < r1; rb += GP_U) {
        float x[GP_U], y[GP_U];
#pragma unroll
        for (int u = 0; u < GP_U; ++u) {
            const int64_t r = rb + u < r1 ? rb + u : r1 - 1;   // rows past the end: not added
            x[u] = a(r);
            y[u] = b(r);
        }
#pragma unroll
        for (int u = 0; u < GP_U; ++u)
            if (rb + u < r1) acc += x[u] * y[u];
    }
    return acc;
}

template <class A>
__device__ __forceinline__ float rows_sum(int64_t r0, int64_t r1, A a)
{
    float acc = 0.0f;
    for (int64_t rb = r0; rb < r1; rb += GP_U) {
        float x[GP_U];
#pragma unroll
        for (int u = 0; u < GP_U; ++u) x[u] = a(rb + u < r1 ? rb + u : r1 - 1);
#pragma unroll
        for (int u = 0; u < GP_U; ++u)
            if (rb + u < r1) acc += x[u];
    }
    return acc;
}

// part[c][p] = sum over the rows of chunk c (in row order) of parameter p's terms
__global__ __launch_bounds__(BLOCK) void k_mlp_grad_parts(const uint16_t *X, int64_t n,
                                                          const uint16_t *h1, const float *h2,
                                                          const float *g, const float *dz2,
                                                          const float *dz1, float *part)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (p >= NPARAM) return;
    const int64_t len = (n + GRAD_CHUNKS - 1) / GRAD_CHUNKS;
    const int64_t r0 = c * len < n ? c * len : n;
    const int64_t r1 = r0 + len < n ? r0 + len : n;
    float acc;
    if (p < OFF_B1) {                       // dW1[j][k] = sum dz1[j] x[k]
        const int j = p / NIN, k = p % NIN;
        acc = rows_dot(r0, r1, [&](int64_t r) { return dz1[r * NH + j]; },
                       [&](int64_t r) { return bf2f(X[r * KP + k]); });
    } else if (p < OFF_W2) {                // db1[j] = sum dz1[j]
        const int j = p - OFF_B1;
        acc = rows_sum(r0, r1, [&](int64_t r) { return dz1[r * NH + j]; });
    } else if (p < OFF_B2) {                // dW2[j][k] = sum dz2[j] h1[k]
        const int j = (p - OFF_W2) / NH, k = (p - OFF_W2) % NH;
        acc = rows_dot(r0, r1, [&](int64_t r) { return dz2[r * NH + j]; },
                       [&](int64_t r) { return bf2f(h1[r * KP + k]); });
    } else if (p < OFF_W3) {                // db2[j] = sum dz2[j]
        const int j = p - OFF_B2;
        acc = rows_sum(r0, r1, [&](int64_t r) { return dz2[r * NH + j]; });
    } else if (p < OFF_B3) {                // dw3[j] = sum g h2[j]
        const int j = p - OFF_W3;
        acc = rows_dot(r0, r1, [&](int64_t r) { return g[r]; },
                       [&](int64_t r) { return h2[r * NH + j]; });
    } else {                                // db3 = sum g
        acc = rows_sum(r0, r1, [&](int64_t r) { return g[r]; });
    }
    part[(int64_t)c * NPARAM + p] = acc;
}

__global__ void k_mlp_grad_reduce(const float *part, float *grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float v[GRAD_CHUNKS];   // all chunks' partials in flight, then added in chunk order
#pragma unroll
    for (int c = 0; c < GRAD_CHUNKS; ++c) v[c] = part[c * NPARAM + p];
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < GRAD_CHUNKS; ++c) acc += v[c];
    grad[p] = acc;
}

// mean of the per-row losses: one block, fixed-order partials and tree
__global__ void k_mlp_loss(const float *loss_rows, int64_t n, float *loss)
{
    __shared__ float part[BLOCK];
    float acc = 0.0f;
    // GP_U rows per thread in flight at once, added in row order
    for (int64_t rb = threadIdx.x; rb < n; rb += (int64_t)GP_U * blockDim.x) {
        float v[GP_U];
#pragma unroll
        for (int u = 0; u < GP_U; ++u) {
            const int64_t r = rb + (int64_t)u * blockDim.x;
            v[u] = r < n ? loss_rows[r] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < GP_U; ++u)
            if (rb + (int64_t)u * blockDim.x < n) acc += v[u];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = n > 0 ? part[0] / (float)n : 0.0f;
}

// Adam with bias correction; c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ void k_mlp_adam(float *P, const float *grad, float *m, float *v, float lr, float b1,
                           float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    const float gr = grad[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gr;
    const float vp = b2 * v[p] + (1.0f - b2) * gr * gr;
    m[p] = mp;
    v[p] = vp;
    P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// ---------------------------------------------------------------- scoring in the chain
struct SmScore {
    MlpW w;
    float mean[NIN], istd[NIN];
    uint16_t x[WAVES][64][LD];
    uint16_t h[WAVES][16][LD];
    float logit[WAVES][64];
    uint32_t pre[NSH + 1];
};

// Every stored object of one kind (triplets or quintuplets): features in
// registers (lane = object), standardised into the wave's LDS tile, four
// 16-row MFMA tiles per wave, then logit and veto (logit below the
// threshold) stored per object.
template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_mlp_score(EvDev E, Consts K, const float *P,
                                                     const float *mean, const float *istd,
                                                     float threshold)
{
    constexpr int NMD = KIND == OT_T3 ? 3 : 5;
    __shared__ SmScore sm;
    if (upstream_overflow(E)) return;
    const uint32_t n = obj_prefix(E, KIND, sm.pre);
    if (blockIdx.x * (WAVES * 64) >= n) return;   // no rows for this block
    load_weights(P, sm.w);
    for (int i = threadIdx.x; i < NIN; i += blockDim.x) {
        sm.mean[i] = mean[i];
        sm.istd[i] = istd[i];
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int k = NIN; k < KP; ++k) sm.x[w][l][k] = 0;   // K padding, never rewritten
    __syncthreads();
    for (uint32_t base = blockIdx.x * (WAVES * 64); base < n; base += gridDim.x * (WAVES * 64)) {
        const uint32_t v = base + w * 64 + l;
        const bool live = v < n;
        const int32_t t = live ? obj_at(E, KIND, sm.pre, v) : 0;
        float f[40];
        if (live) {
            MdV Q[NMD];
            MdX X[NMD];
#pragma unroll
            for (int j = 0; j < NMD; ++j) {
                int32_t m;
                if (KIND == OT_T3) m = j == 0 ? E.t3_a[t] : j == 1 ? E.t3_b[t] : E.t3_c[t];
                else m = t5_md(E, t, j);
                Q[j] = load_md(E, m);
                X[j].bend = E.md_bend[m];
                X[j].is2s = E.md_bar[m] >> 1;
            }
            if constexpr (KIND == OT_T3)
                t3_features(K, Q, X, f);
            else
                t5_features(K, Q, X, tri_curv(Q[0], Q[1], Q[2]), tri_curv(Q[2], Q[3], Q[4]), f);
        } else {
#pragma unroll
            for (int k = 0; k < 40; ++k) f[k] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < NIN; k += 2) {
            const uint32_t lo = f2bf((f[k] - sm.mean[k]) * sm.istd[k]);
            const uint32_t hi = f2bf((f[k + 1] - sm.mean[k + 1]) * sm.istd[k + 1]);
            *reinterpret_cast<uint32_t *>(&sm.x[w][l][k]) = lo | (hi << 16);
        }
        wave_tile_sync();
#pragma unroll 1
        for (int sub = 0; sub < 4; ++sub) {
            float lg[4];
            mlp_tile(sm.w, &sm.x[w][16 * sub], sm.h[w], lg, nullptr, nullptr, 0, 0);
            if ((l & 15) == 0)
#pragma unroll
                for (int r = 0; r < 4; ++r) sm.logit[w][16 * sub + 4 * (l >> 4) + r] = lg[r];
        }
        wave_tile_sync();
        if (live) {
            const float lg = sm.logit[w][l];
            const uint8_t veto = lg >= threshold ? 0 : 1;
            if (KIND == OT_T3) {
                E.t3_logit[t] = lg;
                E.t3_veto[t] = veto;
            } else {
                E.t5_logit[t] = lg;
                E.t5_veto[t] = veto;
            }
        }
    }
}

// ---------------------------------------------------------------- launchers
static int grid_of(int64_t work, int per_block)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > GRID_MAX) g = GRID_MAX;
    return (int)g;
}

size_t mlp_workspace_bytes(int64_t n)
{
    return sizeof(float) * ((size_t)n * (2 + 2 * NH) + (size_t)GRAD_CHUNKS * NPARAM);
}

hipError_t mlp_prepare(const float *F, const float *mean, const float *istd, int64_t n, uint16_t *X,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_prepare, dim3(grid_of(n * KP, BLOCK)), dim3(BLOCK), 0, s, F, mean,
                       istd, n, X);
    return hipGetLastError();
}

hipError_t mlp_forward(const float *P, const uint16_t *X, int64_t n, float *logits, uint16_t *h1,
                       float *h2, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid_of((n + 15) / 16, WAVES)), dim3(BLOCK), 0, s, P, X,
                       n, logits, h1, h2);
    return hipGetLastError();
}

hipError_t mlp_backward(const float *P, const uint16_t *X, const uint8_t *y, int64_t n,
                        const float *logits, const uint16_t *h1, const float *h2, float *work,
                        float *grad, float *loss, hipStream_t s)
{
    float *g = work, *lrow = g + n, *dz2 = lrow + n, *dz1 = dz2 + n * NH, *part = dz1 + n * NH;
    hipLaunchKernelGGL(k_mlp_rows, dim3(grid_of(n, ROWS_PER_BLOCK)), dim3(BLOCK), 0, s, P, logits, y,
                       n, h1, h2, g, dz2, dz1, lrow);
    hipLaunchKernelGGL(k_mlp_grad_parts, dim3((NPARAM + BLOCK - 1) / BLOCK, GRAD_CHUNKS), dim3(BLOCK),
                       0, s, X, n, h1, h2, g, dz2, dz1, part);
    hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((NPARAM + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s,
                       part, grad);
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(BLOCK), 0, s, lrow, n, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------- fixed workspace
// Workspace of the backward pass for callers that cannot allocate: one
// file-scope device array, one copy per GPU, held until the process ends.
// In host code the name `scratch` is only a stand-in for the symbol; its
// device address on each GPU comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is ever passed on.
static __device__ __align__(256) float scratch[MLP_FIXED_SCRATCH_FLOATS];
static_assert(sizeof(float) * ((size_t)MLP_FIXED_MAX_ROWS * (2 + 2 * NH) +
                               (size_t)GRAD_CHUNKS * NPARAM) <= sizeof(scratch),
              "fixed workspace holds MLP_FIXED_MAX_ROWS rows");

static std::mutex scratch_mu;
static void *scratch_at[MLP_FIXED_MAX_DEVICES];

hipError_t mlp_fixed_scratch(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= MLP_FIXED_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_at[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if ((e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t back = hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (back != hipSuccess) return back;
        scratch_at[device] = p;
    }
    *out = scratch_at[device];
    return hipSuccess;
}

hipError_t mlp_adam(float *P, const float *grad, float *m, float *v, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, P, grad,
                       m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_score(const EvDev &E, const Consts &K, int kind, const float *P, const float *mean,
                     const float *istd, float threshold, int grid, hipStream_t s)
{
    if (kind == OT_T3)
        hipLaunchKernelGGL(k_mlp_score<OT_T3>, dim3(grid), dim3(BLOCK), 0, s, E, K, P, mean, istd,
                           threshold);
    else
        hipLaunchKernelGGL(k_mlp_score<OT_T5>, dim3(grid), dim3(BLOCK), 0, s, E, K, P, mean, istd,
                           threshold);
    return hipGetLastError();
}

}  // namespace lst
