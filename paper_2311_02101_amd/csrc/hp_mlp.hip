// Learned initial assignments: per-variable features, a 32 -> 256 -> 1
// perceptron (bfloat16 weights on MFMA, FP32 accumulation) with its training
// kernels (backward with the forward recomputed, a fixed-order reduction of
// its partial sums, Adam), and the initial Bernoulli draws.
//
// Features (per variable, exact dyadic values before one bfloat16 rounding):
//   0..13  clauses of real length l = 1..7 holding the variable positively
//          (index 2(l-1)) / negated (2(l-1)+1), divided by 8
//   14, 15 positive / negated occurrences / 8;  16 their difference / 8
//   17, 18 sum over positive / negated occurrences of 2^-l;  19 difference
//   20..31 zero
// The real length ignores the trailing padding copies of a clause's first
// literal.  Network: q = sigmoid(w2 . relu(W1^T x + b1) + b2).
#include <hip/hip_runtime.h>

#include <cmath>

#include "hp_internal.hpp"
#include "philox.hpp"

namespace hp {

constexpr int kF = HP_MLP_IN;
constexpr int kH = HP_MLP_HIDDEN;
constexpr int kOffW1 = 0, kOffB1 = kF * kH, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH;
constexpr int kFeatAcc = 20;   // accumulated raw features per variable

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    const __bf16 b = (__bf16)x;   // round to nearest even
    return __builtin_bit_cast(uint16_t, b);
}
__device__ __forceinline__ float bf16_value(uint16_t u) {
    return __builtin_bit_cast(float, (uint32_t)u << 16);
}

// formula of a global index, by binary search over prefix offsets [F+1]
__device__ __forceinline__ int formula_of(const int64_t *off, int F, int64_t g) {
    int lo = 0, hi = F;   // off[lo] <= g < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ---- features ----------------------------------------------------------------
__global__ void feature_count_kernel(const uint4 *__restrict__ rec, const int64_t *__restrict__ clause_off,
                                     const FormulaDev *__restrict__ fd, int F, int64_t ctot,
                                     float *__restrict__ acc) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ctot; c += (int64_t)gridDim.x * blockDim.x) {
        const int f = formula_of(clause_off, F, c);
        const int64_t v0 = fd[f].var_off;
        const uint4 r = rec[c];
        const uint32_t e[7] = {r.x & 0xffffu, r.x >> 16, r.y & 0xffffu, r.y >> 16, r.z & 0xffffu, r.z >> 16,
                               r.w & 0xffffu};
        const int len = (int)rec_len(r.w);
        const float jw = ldexpf(1.0f, -len);
        for (int k = 0; k < len; ++k) {
            const int64_t v = v0 + (e[k] & 0x7fffu);
            const int neg = (int)(e[k] >> 15);
            atomicAdd(&acc[v * kFeatAcc + 2 * (len - 1) + neg], 1.0f);
            atomicAdd(&acc[v * kFeatAcc + 14 + neg], 1.0f);
            atomicAdd(&acc[v * kFeatAcc + 17 + neg], jw);
        }
    }
}

__global__ void feature_finish_kernel(const float *__restrict__ acc, int64_t nv, uint16_t *__restrict__ x) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const float *a = acc + v * kFeatAcc;
        float f[kF];
        for (int j = 0; j < 16; ++j) f[j] = a[j] * 0.125f;
        f[16] = (a[14] - a[15]) * 0.125f;
        f[17] = a[17];
        f[18] = a[18];
        f[19] = a[17] - a[18];
        for (int j = 20; j < kF; ++j) f[j] = 0.0f;
        for (int j = 0; j < kF; ++j) x[v * kF + j] = bf16_bits(f[j]);
    }
}

// ---- perceptron: forward -------------------------------------------------------
// One wave per 32-row tile (waves stride over the tiles).  Hidden layer on
// MFMA 32x32x16 bf16: lane l holds rows/columns as
//   A[32 x 16]: row l%32, k = (l/32)*8 + 0..7;  B[16 x 32]: column l%32, same k;
//   D[32 x 32]: register i -> row (i/4)*8 + (l/32)*4 + i%4, column l%32.
constexpr int kWaves = 4;

// row of D register i for lane half h (see above)
__device__ __forceinline__ int d_row(int i, int h) { return (i / 4) * 8 + h * 4 + (i % 4); }

// W1 (transposed bfloat16), b1 and w2 of the network into LDS
__device__ __forceinline__ void load_weights(const float *params, const uint16_t *wbf, uint16_t *s_w1t, float *s_b1,
                                             float *s_w2, int tid) {
    for (int i = tid; i < kH * kF; i += kWaves * 64) s_w1t[i] = wbf[i];
    for (int i = tid; i < kH; i += kWaves * 64) {
        s_b1[i] = params[kOffB1 + i];
        s_w2[i] = bf16_value(wbf[kH * kF + i]);
    }
}

// The two A operands (k-steps) of the 32-row tile starting at row0: lane l
// takes row row0 + l%32, features (l/32)*8 + 0..7 and 16 + (l/32)*8 + 0..7
// (zeros past the last row).  Operands move as integer words: element m of a
// bfloat16 vector is bits 16*(m%2) of word m/2.
__device__ __forceinline__ void load_x_tile(const uint16_t *x, int64_t rows, int64_t row0, int lane, uint4 &x0,
                                            uint4 &x1) {
    const int64_t r = row0 + (lane & 31);
    const int half = lane >> 5;
    x0 = make_uint4(0, 0, 0, 0);
    x1 = make_uint4(0, 0, 0, 0);
    if (r < rows) {
        x0 = *reinterpret_cast<const uint4 *>(x + r * kF + half * 8);
        x1 = *reinterpret_cast<const uint4 *>(x + r * kF + 16 + half * 8);
    }
}

// pre-activations of hidden columns [32 j, 32 j + 32) for the tile's rows
__device__ __forceinline__ f32x16 hidden_chunk(const uint16_t *s_w1t, int j, int lane, bf16x8 a0, bf16x8 a1) {
    const int col = j * 32 + (lane & 31), half = lane >> 5;
    const bf16x8 bw0 = *reinterpret_cast<const bf16x8 *>(s_w1t + col * kF + half * 8);
    const bf16x8 bw1 = *reinterpret_cast<const bf16x8 *>(s_w1t + col * kF + 16 + half * 8);
    f32x16 acc = {};
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, bw0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bw1, acc, 0, 0, 0);
    return acc;
}

// output logits w2 . relu(W1^T x + b1) of the tile's rows, without b2: after
// the butterfly every lane of half h holds s[i] for row d_row(i, h)
__device__ __forceinline__ void tile_logits(const uint16_t *s_w1t, const float *s_b1, const float *s_w2, int lane,
                                            bf16x8 a0, bf16x8 a1, float (&s)[16]) {
    for (int i = 0; i < 16; ++i) s[i] = 0.0f;
    // not unrolled: the unrolled loop hoists every chunk's operand loads and
    // needs twice the registers (half the resident waves) for no gain
#pragma unroll 1
    for (int j = 0; j < 8; ++j) {
        const f32x16 acc = hidden_chunk(s_w1t, j, lane, a0, a1);
        const int col = j * 32 + (lane & 31);
        const float bb = s_b1[col], ww = s_w2[col];
        for (int i = 0; i < 16; ++i) s[i] += fmaxf(acc[i] + bb, 0.0f) * ww;
    }
    for (int off = 1; off < 32; off <<= 1)
        for (int i = 0; i < 16; ++i) s[i] += __shfl_xor(s[i], off, 64);
}

__global__ __launch_bounds__(kWaves * 64) void mlp_forward_kernel(const uint16_t *__restrict__ x, int64_t rows,
                                                                  const float *__restrict__ params,
                                                                  const uint16_t *__restrict__ wbf,
                                                                  float *__restrict__ q_out) {
    __shared__ __align__(16) uint16_t s_w1t[kH * kF];          // W1 transposed: [column][feature]
    __shared__ float s_b1[kH], s_w2[kH];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    load_weights(params, wbf, s_w1t, s_b1, s_w2, tid);
    __syncthreads();
    const float b2 = params[kOffB2];
    const int half = lane >> 5, col_in = lane & 31;
    const int64_t n_tiles = (rows + 31) / 32;
    for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < n_tiles; tile += (int64_t)gridDim.x * kWaves) {
        uint4 x0, x1;
        load_x_tile(x, rows, tile * 32, lane, x0, x1);
        float s[16];
        tile_logits(s_w1t, s_b1, s_w2, lane, __builtin_bit_cast(bf16x8, x0), __builtin_bit_cast(bf16x8, x1), s);
        if (col_in == 0)
            for (int i = 0; i < 16; ++i) {
                const int64_t r = tile * 32 + d_row(i, half);
                if (r < rows) q_out[r] = 1.0f / (1.0f + expf(-(s[i] + b2)));
            }
    }
}

// ---- perceptron: backward --------------------------------------------------------
// A workgroup of 4 waves takes 128 rows per step, as 4 tiles of 32.
//   pass 1: wave w computes the logits of tile w (all 256 hidden columns, as
//           the forward kernel); lanes 0..31 then take one row each for q, the
//           output gradient g = (q - y) / rows and the loss; tile w's rows (row
//           major and transposed) and g go to LDS;
//   pass 2: wave w owns hidden columns [64 w, 64 w + 64) (two MFMA column
//           chunks): for each of the 4 tiles it recomputes their
//           pre-activations, forms dh = g w2 relu'(pre) (bfloat16 for the
//           product) and adds x^T dh to its dW1 chunks, g h to dw2 and dh to db1.
// Each dW1 column is accumulated by one wave only: a wave keeps 2 chunks of
// accumulators instead of all 8 (the register file then holds several waves
// per SIMD), and the workgroup's row of the workspace needs a cross-wave sum
// for b2 and the loss only.  The x^T dh product reuses the D layout as its B
// operand by ordering the reduction index (the rows) as D does:
// step s, k = (l/32)*8 + m  <->  row ((s*8 + m)/4)*8 + (l/32)*4 + m%4.
// (3 waves per SIMD: the register budget of 170 holds pass 2 without spills;
// the compiler's own choice, 2 waves, ran 8% slower)
__global__ __launch_bounds__(kWaves * 64) __attribute__((amdgpu_waves_per_eu(3))) void mlp_backward_kernel(const uint16_t *__restrict__ x,
                                                                   const float *__restrict__ y, int64_t rows,
                                                                   const float *__restrict__ params,
                                                                   const uint16_t *__restrict__ wbf,
                                                                   float *__restrict__ part) {
    __shared__ __align__(16) uint16_t s_w1t[kH * kF];
    __shared__ float s_b1[kH], s_w2[kH];
    __shared__ __align__(16) uint16_t s_x[kWaves][32 * kF];   // tile rows: [row][feature]
    __shared__ __align__(16) uint16_t s_xt[kWaves][kF * 32];  // transposed: [feature][row]
    __shared__ __align__(16) float s_o[kWaves][32];           // logits, then g
    __shared__ float s_red[kWaves][2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    load_weights(params, wbf, s_w1t, s_b1, s_w2, tid);
    __syncthreads();
    const float b2 = params[kOffB2];
    const float inv_rows = 1.0f / (float)rows;
    const int half = lane >> 5, col_in = lane & 31;
    const int64_t n_steps = (rows + 127) / 128;
    f32x16 dw1[2] = {f32x16{}, f32x16{}};
    float dw2[2] = {0.0f, 0.0f}, db1[2] = {0.0f, 0.0f};
    float db2 = 0.0f, lsum = 0.0f;                // lanes 0..31: their rows' sums

    for (int64_t step = blockIdx.x; step < n_steps; step += gridDim.x) {   // uniform over the workgroup
        // ---- pass 1: tile `wave` ----
        const int64_t row0 = (step * kWaves + wave) * 32;
        uint4 x0, x1;
        load_x_tile(x, rows, row0, lane, x0, x1);
        *reinterpret_cast<uint4 *>(&s_x[wave][col_in * kF + half * 8]) = x0;
        *reinterpret_cast<uint4 *>(&s_x[wave][col_in * kF + 16 + half * 8]) = x1;
        {
            const uint32_t w0[4] = {x0.x, x0.y, x0.z, x0.w}, w1[4] = {x1.x, x1.y, x1.z, x1.w};
            for (int m = 0; m < 8; ++m) {
                s_xt[wave][(half * 8 + m) * 32 + col_in] = (uint16_t)(w0[m >> 1] >> (16 * (m & 1)));
                s_xt[wave][(16 + half * 8 + m) * 32 + col_in] = (uint16_t)(w1[m >> 1] >> (16 * (m & 1)));
            }
        }
        float s[16];
        tile_logits(s_w1t, s_b1, s_w2, lane, __builtin_bit_cast(bf16x8, x0), __builtin_bit_cast(bf16x8, x1), s);
        if (col_in == 0)
            for (int q4 = 0; q4 < 4; ++q4)
                *reinterpret_cast<float4 *>(&s_o[wave][q4 * 8 + half * 4]) =
                    make_float4(s[4 * q4] + b2, s[4 * q4 + 1] + b2, s[4 * q4 + 2] + b2, s[4 * q4 + 3] + b2);
        __syncthreads();
        if (lane < 32) {
            const int64_t r = row0 + lane;
            float g = 0.0f;
            if (r < rows) {
                const float o = s_o[wave][lane], yy = y[r];
                const float qq = 1.0f / (1.0f + expf(-o));
                g = (qq - yy) * inv_rows;
                // softplus(o) - y o
                const float sp = o > 0.0f ? o + log1pf(expf(-o)) : log1pf(expf(o));
                lsum += sp - yy * o;
                db2 += g;
            }
            s_o[wave][lane] = g;
        }
        __syncthreads();
        // ---- pass 2: columns of chunks 2 wave, 2 wave + 1 over the 4 tiles ----
        for (int t = 0; t < kWaves; ++t) {
            const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(&s_x[t][col_in * kF + half * 8]);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(&s_x[t][col_in * kF + 16 + half * 8]);
            uint32_t t0[4], t1[4];   // x^T with rows in the D-register order
            for (int m = 0; m < 8; m += 2) {
                const int r0 = d_row(m, half), r1 = d_row(8 + m, half);
                t0[m >> 1] = *reinterpret_cast<const uint32_t *>(&s_xt[t][col_in * 32 + r0]);
                t1[m >> 1] = *reinterpret_cast<const uint32_t *>(&s_xt[t][col_in * 32 + r1]);
            }
            const bf16x8 ax0 = __builtin_bit_cast(bf16x8, make_uint4(t0[0], t0[1], t0[2], t0[3]));
            const bf16x8 ax1 = __builtin_bit_cast(bf16x8, make_uint4(t1[0], t1[1], t1[2], t1[3]));
            float g[16];
            for (int q4 = 0; q4 < 4; ++q4) {
                const float4 v = *reinterpret_cast<const float4 *>(&s_o[t][q4 * 8 + half * 4]);
                g[4 * q4] = v.x;
                g[4 * q4 + 1] = v.y;
                g[4 * q4 + 2] = v.z;
                g[4 * q4 + 3] = v.w;
            }
            for (int c = 0; c < 2; ++c) {
                const int j = 2 * wave + c, col = j * 32 + col_in;
                const f32x16 acc = hidden_chunk(s_w1t, j, lane, a0, a1);
                const float bb = s_b1[col], ww = s_w2[col];
                uint32_t dq[8];
                for (int i = 0; i < 16; ++i) {
                    const float pre = acc[i] + bb;
                    dw2[c] += g[i] * fmaxf(pre, 0.0f);
                    const float dh = pre > 0.0f ? g[i] * ww : 0.0f;
                    db1[c] += dh;
                    const uint32_t bits = bf16_bits(dh);
                    dq[i >> 1] = (i & 1) ? (dq[i >> 1] | (bits << 16)) : bits;
                }
                const bf16x8 d0 = __builtin_bit_cast(bf16x8, make_uint4(dq[0], dq[1], dq[2], dq[3]));
                const bf16x8 d1 = __builtin_bit_cast(bf16x8, make_uint4(dq[4], dq[5], dq[6], dq[7]));
                dw1[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ax0, d0, dw1[c], 0, 0, 0);
                dw1[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ax1, d1, dw1[c], 0, 0, 0);
            }
        }
        __syncthreads();                                // before the next step's tiles overwrite LDS
    }
    // ---- the workgroup's row of the workspace (plain stores) ----
    float *row = part + (size_t)blockIdx.x * (HP_MLP_PARAMS + 1);
    for (int c = 0; c < 2; ++c) {
        const int col = (2 * wave + c) * 32 + col_in;
        for (int i = 0; i < 16; ++i) row[kOffW1 + d_row(i, half) * kH + col] = dw1[c][i];
        // both halves of the wave hold partials of column col
        const float w2s = dw2[c] + __shfl_xor(dw2[c], 32, 64);
        const float b1s = db1[c] + __shfl_xor(db1[c], 32, 64);
        if (half == 0) {
            row[kOffW2 + col] = w2s;
            row[kOffB1 + col] = b1s;
        }
    }
    // b2 and the loss: a fixed butterfly over the wave, then the waves in order
    for (int off = 1; off < 64; off <<= 1) {
        db2 += __shfl_xor(db2, off, 64);
        lsum += __shfl_xor(lsum, off, 64);
    }
    if (lane == 0) {
        s_red[wave][0] = db2;
        s_red[wave][1] = lsum;
    }
    __syncthreads();
    if (tid == 0) {
        float b = s_red[0][0], l = s_red[0][1];
        for (int w = 1; w < kWaves; ++w) {
            b += s_red[w][0];
            l += s_red[w][1];
        }
        row[kOffB2] = b;
        row[HP_MLP_PARAMS] = l;
    }
}

// grad[p] (p < HP_MLP_PARAMS) and the loss (p = HP_MLP_PARAMS) = the sum of
// column p over the workspace's first `parts` rows, in a fixed order: 16 row
// groups per column summed by 16 waves, then the groups in order.  A wave
// reads 64 consecutive columns of a row (256 bytes) per load.
__global__ __launch_bounds__(1024) void mlp_reduce_kernel(const float *__restrict__ part, int parts,
                                                          float *__restrict__ grad, float *__restrict__ loss_sum) {
    __shared__ float s[16][64];
    const int c = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + c;
    const int per = (parts + 15) / 16, lo = grp * per, hi = min(parts, lo + per);
    float sum = 0.0f;
    if (p <= HP_MLP_PARAMS)
        for (int b = lo; b < hi; ++b) sum += part[(size_t)b * (HP_MLP_PARAMS + 1) + p];
    s[grp][c] = sum;
    __syncthreads();
    if (grp == 0 && p <= HP_MLP_PARAMS) {
        float t = s[0][c];
        for (int k = 1; k < 16; ++k) t += s[k][c];
        if (p < HP_MLP_PARAMS) grad[p] = t;
        else *loss_sum = t;
    }
}

// ---- Adam and the bfloat16 weight copies --------------------------------------
__global__ void adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, float lr, float beta1, float beta2, float eps,
                            float corr1, float corr2, uint16_t *__restrict__ wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= HP_MLP_PARAMS) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / corr1) / (sqrtf(vi / corr2) + eps);
    p[i] = pi;
    if (i < kOffB1) {
        const int f = i / kH, col = i % kH;
        wbf[col * kF + f] = bf16_bits(pi);
    } else if (i >= kOffW2 && i < kOffB2) {
        wbf[kH * kF + (i - kOffW2)] = bf16_bits(pi);
    }
}

__global__ void weights_to_bf16_kernel(const float *__restrict__ p, uint16_t *__restrict__ wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kOffB1) {
        const int f = i / kH, col = i % kH;
        wbf[col * kF + f] = bf16_bits(p[i]);
    } else if (i >= kOffW2 && i < kOffB2) {
        wbf[kH * kF + (i - kOffW2)] = bf16_bits(p[i]);
    }
}

__global__ void zero_f32_kernel(float *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// ---- initial assignments v = [U < q] at the reserved time 2^64 - 1 -------------
__global__ void init_chains_kernel(const float *__restrict__ q, const int64_t *__restrict__ var_off, int F,
                                   int64_t nv, int B, int chain_lo, uint32_t key0, uint32_t key1,
                                   uint8_t *__restrict__ v) {
    const int b = chain_lo + blockIdx.y;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < nv; g += (int64_t)gridDim.x * blockDim.x) {
        const int f = formula_of(var_off, F, g);
        const int64_t i = g - var_off[f];
        const int64_t n = var_off[f + 1] - var_off[f];
        const uint4 r = philox4x32_10_lane_key(
            make_uint4(0xffffffffu, (uint32_t)b, kPhaseVisible | (uint32_t)(i >> 2), 0xffffffffu),
            Key2{key0, key1 ^ (uint32_t)f});
        const uint32_t w = (i & 3) == 0 ? r.x : (i & 3) == 1 ? r.y : (i & 3) == 2 ? r.z : r.w;
        const float u = (float)(w >> 8) * (1.0f / 16777216.0f);
        v[var_off[f] * B + (int64_t)b * n + i] = u < q[g] ? 1 : 0;
    }
}

// ---- per-variable mean over the chains of a state-layout byte array -------------
__global__ void chain_mean_kernel(const uint8_t *__restrict__ a, const int64_t *__restrict__ var_off, int F,
                                  int64_t nv, int B, float *__restrict__ out) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < nv; g += (int64_t)gridDim.x * blockDim.x) {
        const int f = formula_of(var_off, F, g);
        const int64_t i = g - var_off[f], n = var_off[f + 1] - var_off[f];
        int s = 0;
        for (int b = 0; b < B; ++b) s += a[var_off[f] * B + (int64_t)b * n + i];
        out[g] = (float)s / (float)B;
    }
}

// ---- launchers --------------------------------------------------------------
static int grid_for(int64_t n, int per_block, int cap) {
    const int64_t g = (n + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

hipError_t launch_features(const Plan &p, float *acc, uint16_t *x, hipStream_t s) {
    zero_f32_kernel<<<grid_for(p.total_vars * kFeatAcc, 256, 4096), 256, 0, s>>>(acc, p.total_vars * kFeatAcc);
    feature_count_kernel<<<grid_for(p.total_clauses, 256, 8192), 256, 0, s>>>(p.d_rec, p.d_clause_off, p.d_fd, p.F,
                                                                             p.total_clauses, acc);
    feature_finish_kernel<<<grid_for(p.total_vars, 256, 8192), 256, 0, s>>>(acc, p.total_vars, x);
    return hipGetLastError();
}

hipError_t launch_mlp(const hp_mlp &net, const uint16_t *x, const float *y, int64_t rows, float *q, float *loss_sum,
                      bool backward, hipStream_t s) {
    if (backward) {
        // 128 rows per workgroup step; one workspace row per workgroup
        const int grid = grid_for((rows + 127) / 128, 1, HP_MLP_PARTS);
        mlp_backward_kernel<<<grid, kWaves * 64, 0, s>>>(x, y, rows, net.params, net.w_bf16, net.partials);
        mlp_reduce_kernel<<<(HP_MLP_PARAMS + 1 + 63) / 64, 1024, 0, s>>>(net.partials, grid, net.grad, loss_sum);
    } else {
        const int grid = grid_for((rows + 31) / 32, kWaves, 1024);
        mlp_forward_kernel<<<grid, kWaves * 64, 0, s>>>(x, rows, net.params, net.w_bf16, q);
    }
    return hipGetLastError();
}

hipError_t launch_adam(const hp_mlp &net, float lr, float beta1, float beta2, float eps, int64_t step, hipStream_t s) {
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    adam_kernel<<<(HP_MLP_PARAMS + 255) / 256, 256, 0, s>>>(net.params, net.adam_m, net.adam_v, net.grad, lr, beta1,
                                                           beta2, eps, c1, c2, net.w_bf16);
    return hipGetLastError();
}

hipError_t launch_weights_to_bf16(const hp_mlp &net, hipStream_t s) {
    weights_to_bf16_kernel<<<(kOffB2 + 255) / 256, 256, 0, s>>>(net.params, net.w_bf16);
    return hipGetLastError();
}

hipError_t launch_init_chains(const Plan &p, const float *q, int chain_lo, int chain_hi, uint8_t *v, hipStream_t s) {
    if (chain_hi <= chain_lo) return hipSuccess;
    dim3 grid(grid_for(p.total_vars, 256, 1024), chain_hi - chain_lo);
    init_chains_kernel<<<grid, 256, 0, s>>>(q, p.d_var_off, p.F, p.total_vars, p.B, chain_lo,
                                            (uint32_t)(p.seed & 0xffffffffu), (uint32_t)(p.seed >> 32), v);
    return hipGetLastError();
}

hipError_t launch_chain_mean(const Plan &p, const uint8_t *a, float *out, hipStream_t s) {
    chain_mean_kernel<<<grid_for(p.total_vars, 256, 8192), 256, 0, s>>>(a, p.d_var_off, p.F, p.total_vars, p.B, out);
    return hipGetLastError();
}

}  // namespace hp
