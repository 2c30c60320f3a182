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
// Training uses the same forward tile (saving the hidden activations, or
// fused into the gradient kernel), a backward pass whose products run on the
// matrix cores in FP32 (v_mfma_f32_16x16x4_f32) per chunk of rows, followed
// by a reduction over the chunks in a fixed order (gradients are bit-for-bit
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
// are stored.  A and H are the calling wave's own tiles.  If h2v is given,
// lane l receives the second hidden layer's units 16 nt + l%16 of rows
// 4 (l/16) + r in h2v[nt][r], and every lane the logits of its rows.
__device__ __forceinline__ void mlp_tile(const MlpW &w, const uint16_t (*A)[LD], uint16_t (*H)[LD],
                                         float logit[4], uint16_t *h1_out, float *h2_out,
                                         int64_t row0, int64_t n, float (*h2v)[4] = nullptr)
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
            if (h2v) h2v[nt][r] = h2;
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
// Gradient of the mean BCE-with-logits loss from the row terms
//   g = (sigmoid(z) - y) / n,  dz2 = g w3 [h2 > 0],  dz1 = (dz2 W2) [h1 > 0]
// (W2 the BF16-rounded weights the forward used), summed over the rows:
//   dW1 = dz1^T X, db1 = sum dz1, dW2 = dz2^T h1, db2 = sum dz2,
//   dw3 = h2^T g, db3 = sum g.
// The rows split into at most GRAD_CHUNKS chunks of whole 64-row batches,
// one block per chunk.  In each batch a wave takes 16 rows: their forward
// (FWD) or the stored logits and hidden layers, the row terms into LDS, and
// dz1 as a 16 x 64 x 64 FP32 matrix product.  The block's waves then share
// the 28 16 x 16 tiles of dW1 (64 x 48, inputs zero padded) and dW2
// (64 x 64), each a product over the batch's 64 rows; their accumulators
// stay in registers over the chunk's batches.  Products are FP32 matrix-core
// steps (v_mfma_f32_16x16x4_f32: lane l supplies A[l%16][l/16] and
// B[l/16][l%16], receives D rows 4 (l/16) + r, column l%16).  The vector
// sums are kept per lane over its rows and combined in a fixed order at the
// end.  A block writes its chunk's partial gradient; k_mlp_reduce adds the
// chunks in chunk order.  Every sum runs in an order fixed by n alone, so the
// gradient is bit-for-bit reproducible, and the forward-fused and the
// stored-activation variants give the same bits.
constexpr int RB = WAVES * 16;     // rows per batch of a block
// row stride of the FP32 row-term tiles: the gradient products read 16
// consecutive columns of 4 consecutive rows per instruction, which a stride
// of 16 banks (mod 64) spreads over distinct banks
constexpr int DS = NH + 16;
constexpr int GT = 28;             // gradient tiles: 12 of dW1, 16 of dW2
constexpr int GT_W = GT / WAVES;   // per wave
static_assert(GT % WAVES == 0 && NIN <= 48, "gradient tiles");

struct SmGrad {
    MlpW w;
    uint16_t x[WAVES][16][LD];     // inputs (BF16)
    uint16_t h[WAVES][16][LD];     // first hidden layer (BF16)
    float d2[WAVES][16][DS];       // dz2
    float d1[WAVES][16][DS];       // dz1
    float vs[WAVES][3][NH];        // the waves' db1, db2, dw3
    float gs[WAVES];               // the waves' db3
};

__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// rows of the chunk c: [c clen, min((c + 1) clen, n)), clen a multiple of RB
static void grad_chunks(int64_t n, int &nch, int64_t &clen)
{
    int64_t b = (n + RB - 1) / RB;
    if (b < 1) b = 1;
    nch = (int)(b < GRAD_CHUNKS ? b : GRAD_CHUNKS);
    clen = (b + nch - 1) / nch * RB;
}

template <bool FWD>
__global__ __launch_bounds__(BLOCK) void k_mlp_grad(const float *P, const uint16_t *X,
                                                    const uint8_t *y, int64_t n, int64_t clen,
                                                    const float *logits, const uint16_t *h1,
                                                    const float *h2, float *loss_rows, float *part)
{
    __shared__ SmGrad sm;
    load_weights(P, sm.w);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int col = l & 15, q = l >> 4, rq = 4 * q;
    const int64_t r0 = (int64_t)blockIdx.x * clen;
    const int64_t r1 = r0 + clen < n ? r0 + clen : n;
    f32x4 acc[GT_W];
#pragma unroll
    for (int i = 0; i < GT_W; ++i) acc[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float sb1[4] = {0.0f, 0.0f, 0.0f, 0.0f}, sb2[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float sw3[4] = {0.0f, 0.0f, 0.0f, 0.0f}, sg = 0.0f;
    // operands of the wave's gradient tiles: column 16 jt + l%16 of dz1 (dW1)
    // or dz2 (dW2) and column 16 kt + l%16 of the inputs or h1, at row 0
    const float *ta[GT_W];
    const uint16_t *tb[GT_W];
#pragma unroll
    for (int i = 0; i < GT_W; ++i) {
        const int t = w + WAVES * i;
        const bool first = t < 12;
        const int jt = first ? t / 3 : (t - 12) / 4, kt = first ? t % 3 : (t - 12) % 4;
        ta[i] = (first ? &sm.d1[0][0][0] : &sm.d2[0][0][0]) + 16 * jt + col;
        tb[i] = (first ? &sm.x[0][0][0] : &sm.h[0][0][0]) + 16 * kt + col;
    }
    __syncthreads();   // weights staged
    for (int64_t b0 = r0; b0 < r1; b0 += RB) {
        const int64_t row0 = b0 + 16 * w;
        // the wave's 16 input rows (and stored first hidden layer), zero past the chunk
        for (int i = l; i < 16 * (KP / 8); i += 64) {
            const int r = i / (KP / 8), c8 = (i % (KP / 8)) * 8;
            uint4 v = make_uint4(0u, 0u, 0u, 0u), u = v;
            if (row0 + r < r1) {
                v = *reinterpret_cast<const uint4 *>(&X[(row0 + r) * KP + c8]);
                if (!FWD) u = *reinterpret_cast<const uint4 *>(&h1[(row0 + r) * KP + c8]);
            }
            *reinterpret_cast<uint4 *>(&sm.x[w][r][c8]) = v;
            if (!FWD) *reinterpret_cast<uint4 *>(&sm.h[w][r][c8]) = u;
        }
        wave_tile_sync();
        float lg[4], h2v[4][4];
        if (FWD) {
            mlp_tile(sm.w, sm.x[w], sm.h[w], lg, nullptr, nullptr, row0, r1, h2v);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + rq + r;
                const bool live = row < r1;
                lg[r] = live ? logits[row] : 0.0f;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) h2v[nt][r] = live ? h2[row * NH + 16 * nt + col] : 0.0f;
            }
        }
        // row terms: g, the loss per row, dz2 (lane: units 16 nt + col of rows rq + r)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + rq + r;
            const bool live = row < r1;
            const float z = lg[r];
            const float yv = live && y[row] ? 1.0f : 0.0f;
            const float gr = live ? (1.0f / (1.0f + expf(-z)) - yv) / (float)n : 0.0f;
            if (live && col == 0)
                loss_rows[row] = (z > 0.0f ? z : 0.0f) - z * yv + log1pf(expf(-fabsf(z)));
            if (col == 0) sg += gr;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int j = 16 * nt + col;
                const float dj = h2v[nt][r] > 0.0f ? gr * sm.w.w3[j] : 0.0f;
                sm.d2[w][rq + r][j] = dj;
                sb2[nt] += dj;
                sw3[nt] += gr * h2v[nt][r];
            }
        }
        wave_tile_sync();
        // dz1 (16 x 64) = dz2 (16 x 64) W2 (64 x 64), masked where h1 is zero
        {
            f32x4 d[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) d[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < NH / 4; ++ks) {
                const float a = sm.d2[w][col][4 * ks + q];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    d[nt] = mfma_f32(a, bf2f(sm.w.w2[4 * ks + q][16 * nt + col]), d[nt]);
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = 16 * nt + col;
                    const float v = sm.h[w][rq + r][j] != 0 ? d[nt][r] : 0.0f;
                    sm.d1[w][rq + r][j] = v;
                    sb1[nt] += v;
                }
        }
        __syncthreads();   // every wave's rows in LDS
        // the wave's gradient tiles t = w + WAVES i over the batch's 64 rows,
        // four rows per step; the tiles' products of one step are independent
#pragma unroll 2
        for (int s = 0; s < RB / 4; ++s) {
            const int row = 4 * s + q;
#pragma unroll
            for (int i = 0; i < GT_W; ++i)
                acc[i] = mfma_f32(ta[i][row * DS], bf2f(tb[i][row * LD]), acc[i]);
        }
        __syncthreads();   // the tiles are rewritten by the next batch
    }
    // the chunk's partial gradient
    float *pc = part + (int64_t)blockIdx.x * NPARAM;
#pragma unroll
    for (int i = 0; i < GT_W; ++i) {
        const int t = w + WAVES * i;
        const bool first = t < 12;
        const int jt = first ? t / 3 : (t - 12) / 4, kt = first ? t % 3 : (t - 12) % 4;
        const int k = 16 * kt + col;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = 16 * jt + rq + r;
            if (first) {
                if (k < NIN) pc[OFF_W1 + j * NIN + k] = acc[i][r];
            } else {
                pc[OFF_W2 + j * NH + k] = acc[i][r];
            }
        }
    }
    // vector sums: the four row quarters of the wave, then the waves in order
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        float a = sb1[nt], b = sb2[nt], c = sw3[nt];
        a += __shfl_xor(a, 16, 64);
        b += __shfl_xor(b, 16, 64);
        c += __shfl_xor(c, 16, 64);
        a += __shfl_xor(a, 32, 64);
        b += __shfl_xor(b, 32, 64);
        c += __shfl_xor(c, 32, 64);
        if (q == 0) {
            sm.vs[w][0][16 * nt + col] = a;
            sm.vs[w][1][16 * nt + col] = b;
            sm.vs[w][2][16 * nt + col] = c;
        }
    }
    sg += __shfl_xor(sg, 16, 64);
    sg += __shfl_xor(sg, 32, 64);
    if (l == 0) sm.gs[w] = sg;
    __syncthreads();
    const int tid = threadIdx.x;
    if (tid < 3 * NH) {
        const int v = tid / NH, j = tid % NH;
        float a = 0.0f;
#pragma unroll
        for (int ww = 0; ww < WAVES; ++ww) a += sm.vs[ww][v][j];
        pc[(v == 0 ? OFF_B1 : v == 1 ? OFF_B2 : OFF_W3) + j] = a;
    } else if (tid == 3 * NH) {
        float a = 0.0f;
#pragma unroll
        for (int ww = 0; ww < WAVES; ++ww) a += sm.gs[ww];
        pc[OFF_B3] = a;
    }
}

// mean of the per-row losses: one block, fixed-order partials and tree;
// GP_U rows per thread are loaded before they are added
constexpr int GP_U = 16;

// mean of the per-row losses: one block, fixed-order partials and tree
__device__ __forceinline__ void loss_body(const float *loss_rows, int64_t n, float *loss)
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
struct AdamArgs {
    float *m, *v;
    float lr, b1, b2, eps, c1, c2;
};

__device__ __forceinline__ void adam_one(float *P, int p, float gr, const AdamArgs &a)
{
    const float mp = a.b1 * a.m[p] + (1.0f - a.b1) * gr;
    const float vp = a.b2 * a.v[p] + (1.0f - a.b2) * gr * gr;
    a.m[p] = mp;
    a.v[p] = vp;
    P[p] -= a.lr * (mp / a.c1) / (sqrtf(vp / a.c2) + a.eps);
}

__global__ void k_mlp_adam(float *P, const float *grad, AdamArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    adam_one(P, p, grad[p], a);
}

// The end of a backward pass in one launch: grad[p] is the sum of the
// chunks' partials in chunk order, followed (ADAM) by the Adam update of
// parameter p with the same operations as k_mlp_adam; the block past the
// parameters takes the mean loss (loss_body).
template <bool ADAM>
__global__ void k_mlp_reduce(const float *part, int nch, float *grad, const float *loss_rows,
                             int64_t n, float *loss, float *P, AdamArgs a)
{
    if (blockIdx.x == gridDim.x - 1) {
        loss_body(loss_rows, n, loss);
        return;
    }
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float v[GRAD_CHUNKS];   // all chunks' partials in flight, then added in chunk order
#pragma unroll
    for (int c = 0; c < GRAD_CHUNKS; ++c) v[c] = c < nch ? part[c * NPARAM + p] : 0.0f;
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < GRAD_CHUNKS; ++c)
        if (c < nch) acc += v[c];
    grad[p] = acc;
    if (ADAM) adam_one(P, p, acc, a);
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

// backward workspace: the per-row losses, then the chunks' partial gradients
size_t mlp_workspace_bytes(int64_t n)
{
    return sizeof(float) * ((size_t)n + (size_t)GRAD_CHUNKS * NPARAM);
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
    float *lrow = work, *part = work + n;
    int nch;
    int64_t clen;
    grad_chunks(n, nch, clen);
    hipLaunchKernelGGL(k_mlp_grad<false>, dim3(nch), dim3(BLOCK), 0, s, P, X, y, n, clen, logits, h1,
                       h2, lrow, part);
    // the chunk sums and the mean loss in one launch (the loss in the last block)
    hipLaunchKernelGGL(k_mlp_reduce<false>, dim3((NPARAM + BLOCK - 1) / BLOCK + 1), dim3(BLOCK), 0, s,
                       part, nch, grad, lrow, n, loss, nullptr, AdamArgs{});
    return hipGetLastError();
}

// One Adam step on n rows in two launches, with the same operations in the
// same order as mlp_forward, mlp_backward and mlp_adam one after the other:
// the forward fused with the per-chunk gradient products, then the chunk
// reduction with the Adam update and the mean loss.
hipError_t mlp_train_step(float *P, const uint16_t *X, const uint8_t *y, int64_t n, float *work,
                          float *grad, float *loss, float *m, float *v, float lr, float b1, float b2,
                          float eps, float c1, float c2, hipStream_t s)
{
    float *lrow = work, *part = work + n;
    int nch;
    int64_t clen;
    grad_chunks(n, nch, clen);
    hipLaunchKernelGGL(k_mlp_grad<true>, dim3(nch), dim3(BLOCK), 0, s, P, X, y, n, clen, nullptr,
                       nullptr, nullptr, lrow, part);
    hipLaunchKernelGGL(k_mlp_reduce<true>, dim3((NPARAM + BLOCK - 1) / BLOCK + 1), dim3(BLOCK), 0, s,
                       part, nch, grad, lrow, n, loss, P, AdamArgs{m, v, lr, b1, b2, eps, c1, c2});
    return hipGetLastError();
}

// ---------------------------------------------------------------- fixed workspace
// Workspace of the backward pass for callers that cannot allocate: one
// file-scope device array, one copy per GPU, held until the process ends.
// In host code the name `scratch` is only a stand-in for the symbol; its
// device address on each GPU comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is ever passed on.
static __device__ __align__(256) float scratch[MLP_FIXED_SCRATCH_FLOATS];
static_assert(sizeof(float) * ((size_t)MLP_FIXED_MAX_ROWS + (size_t)GRAD_CHUNKS * NPARAM) <=
                  sizeof(scratch),
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
                       AdamArgs{m, v, lr, b1, b2, eps, c1, c2});
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
