// Learned initial assignments: per-variable features, a 32 -> 256 -> 1
// perceptron (bfloat16 weights on MFMA, FP32 accumulation) with its training
// kernels (forward + backward fused, Adam), and the initial Bernoulli draws.
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
        const int len = (int)((r.w >> 16) & 7u);
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

// ---- perceptron: forward (+ backward) ------------------------------------------
// One wave per 32-row tile (waves stride over the tiles).  Hidden layer on
// MFMA 32x32x16 bf16: lane l holds rows/columns as
//   A[32 x 16]: row l%32, k = (l/32)*8 + 0..7;  B[16 x 32]: column l%32, same k;
//   D[32 x 32]: register i -> row (i/4)*8 + (l/32)*4 + i%4, column l%32.
// The backward product dW1 = x^T dh reuses each lane's own D registers as the
// B operand by ordering its reduction index (the rows) as the D layout does:
// step s, k = (l/32)*8 + m  <->  row ((s*8 + m)/4)*8 + (l/32)*4 + m%4.
constexpr int kWaves = 4;

template <bool kBackward>
__global__ __launch_bounds__(kWaves * 64) void mlp_kernel(const uint16_t *__restrict__ x, const float *__restrict__ y,
                                                          int64_t rows, const float *__restrict__ params,
                                                          const uint16_t *__restrict__ wbf, float *__restrict__ q_out,
                                                          float *__restrict__ grad, float *__restrict__ loss_sum) {
    __shared__ __align__(16) uint16_t s_w1t[kH * kF];          // W1 transposed: [column][feature]
    __shared__ float s_b1[kH], s_w2[kH];
    __shared__ __align__(16) uint16_t s_xt[kWaves][kF * 32];   // x tile transposed: [feature][row]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < kH * kF; i += blockDim.x) s_w1t[i] = wbf[i];
    for (int i = tid; i < kH; i += blockDim.x) {
        s_b1[i] = params[kOffB1 + i];
        s_w2[i] = bf16_value(wbf[kH * kF + i]);
    }
    __syncthreads();
    const float b2 = params[kOffB2];
    const float inv_rows = 1.0f / (float)rows;
    const int half = lane >> 5, col_in = lane & 31;
    const int64_t n_tiles = (rows + 31) / 32;
    f32x16 dw1[8];
    float dw2[8], db1[8];
    for (int j = 0; j < 8; ++j) {
        dw1[j] = f32x16{};
        dw2[j] = 0.0f;
        db1[j] = 0.0f;
    }
    float db2 = 0.0f, lsum = 0.0f;

    for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < n_tiles; tile += (int64_t)gridDim.x * kWaves) {
        // ---- load the x tile (A operands of the two k-steps) ----
        // operands move as integer words: element m of a bfloat16 vector is
        // bits 16*(m%2) of word m/2
        const int64_t row_a = tile * 32 + col_in;
        uint4 x0 = make_uint4(0, 0, 0, 0), x1 = make_uint4(0, 0, 0, 0);
        if (row_a < rows) {
            x0 = *reinterpret_cast<const uint4 *>(x + row_a * kF + half * 8);
            x1 = *reinterpret_cast<const uint4 *>(x + row_a * kF + 16 + half * 8);
        }
        const bf16x8 a0 = __builtin_bit_cast(bf16x8, x0), a1 = __builtin_bit_cast(bf16x8, x1);
        if (kBackward) {
            const uint32_t w0[4] = {x0.x, x0.y, x0.z, x0.w}, w1[4] = {x1.x, x1.y, x1.z, x1.w};
            for (int m = 0; m < 8; ++m) {
                s_xt[wave][(half * 8 + m) * 32 + col_in] = (uint16_t)(w0[m >> 1] >> (16 * (m & 1)));
                s_xt[wave][(16 + half * 8 + m) * 32 + col_in] = (uint16_t)(w1[m >> 1] >> (16 * (m & 1)));
            }
        }
        // ---- pass 1: output logit of every row ----
        float s[16];
        for (int i = 0; i < 16; ++i) s[i] = 0.0f;
        for (int j = 0; j < 8; ++j) {
            const int col = j * 32 + col_in;
            const bf16x8 bw0 = *reinterpret_cast<const bf16x8 *>(s_w1t + col * kF + half * 8);
            const bf16x8 bw1 = *reinterpret_cast<const bf16x8 *>(s_w1t + col * kF + 16 + half * 8);
            f32x16 acc = {};
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, bw0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bw1, acc, 0, 0, 0);
            const float bb = s_b1[col], ww = s_w2[col];
            for (int i = 0; i < 16; ++i) s[i] += fmaxf(acc[i] + bb, 0.0f) * ww;
        }
        for (int off = 1; off < 32; off <<= 1)
            for (int i = 0; i < 16; ++i) s[i] += __shfl_xor(s[i], off, 64);
        float o[16], g[16];
        for (int i = 0; i < 16; ++i) {
            const int64_t r = tile * 32 + (i / 4) * 8 + half * 4 + (i % 4);
            o[i] = s[i] + b2;
            const float qq = 1.0f / (1.0f + expf(-o[i]));
            if (!kBackward) {
                if (col_in == 0 && r < rows) q_out[r] = qq;
            } else {
                float yy = 0.0f;
                if (r < rows) yy = y[r];
                g[i] = r < rows ? (qq - yy) * inv_rows : 0.0f;
                if (col_in == 0 && r < rows) {
                    // softplus(o) - y o
                    const float sp = o[i] > 0.0f ? o[i] + log1pf(expf(-o[i])) : log1pf(expf(o[i]));
                    lsum += sp - yy * o[i];
                    db2 += g[i];
                }
            }
        }
        if (!kBackward) continue;
        // ---- pass 2: hidden-layer gradients ----
        __builtin_amdgcn_wave_barrier();
        uint32_t t0[4], t1[4];   // x^T with rows in the D-register order
        for (int m = 0; m < 8; m += 2) {
            const int r0 = (m / 4) * 8 + half * 4 + (m % 4);          // step 0: i = m, m + 1
            const int r1 = ((8 + m) / 4) * 8 + half * 4 + (m % 4);    // step 1: i = 8 + m, 9 + m
            t0[m >> 1] = (uint32_t)s_xt[wave][col_in * 32 + r0] | ((uint32_t)s_xt[wave][col_in * 32 + r0 + 1] << 16);
            t1[m >> 1] = (uint32_t)s_xt[wave][col_in * 32 + r1] | ((uint32_t)s_xt[wave][col_in * 32 + r1 + 1] << 16);
        }
        const bf16x8 ax0 = __builtin_bit_cast(bf16x8, make_uint4(t0[0], t0[1], t0[2], t0[3]));
        const bf16x8 ax1 = __builtin_bit_cast(bf16x8, make_uint4(t1[0], t1[1], t1[2], t1[3]));
        for (int j = 0; j < 8; ++j) {
            const int col = j * 32 + col_in;
            const bf16x8 bw0 = *reinterpret_cast<const bf16x8 *>(s_w1t + col * kF + half * 8);
            const bf16x8 bw1 = *reinterpret_cast<const bf16x8 *>(s_w1t + col * kF + 16 + half * 8);
            f32x16 acc = {};
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, bw0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bw1, acc, 0, 0, 0);
            const float bb = s_b1[col], ww = s_w2[col];
            uint32_t dq[8];
            for (int i = 0; i < 16; ++i) {
                const float pre = acc[i] + bb;
                const float h = fmaxf(pre, 0.0f);
                dw2[j] += g[i] * h;
                const float dh = pre > 0.0f ? g[i] * ww : 0.0f;
                db1[j] += dh;
                const uint32_t bits = bf16_bits(dh);
                dq[i >> 1] = (i & 1) ? (dq[i >> 1] | (bits << 16)) : bits;
            }
            const bf16x8 d0 = __builtin_bit_cast(bf16x8, make_uint4(dq[0], dq[1], dq[2], dq[3]));
            const bf16x8 d1 = __builtin_bit_cast(bf16x8, make_uint4(dq[4], dq[5], dq[6], dq[7]));
            dw1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ax0, d0, dw1[j], 0, 0, 0);
            dw1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ax1, d1, dw1[j], 0, 0, 0);
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (!kBackward) return;
    // ---- reduce this wave's gradient partials into the global buffer ----
    for (int j = 0; j < 8; ++j) {
        const int col = j * 32 + col_in;
        for (int i = 0; i < 16; ++i) {
            const int f = (i / 4) * 8 + half * 4 + (i % 4);
            atomicAdd(&grad[kOffW1 + f * kH + col], dw1[j][i]);
        }
        const float w2s = dw2[j] + __shfl_xor(dw2[j], 32, 64);
        const float b1s = db1[j] + __shfl_xor(db1[j], 32, 64);
        if (half == 0) {
            atomicAdd(&grad[kOffW2 + col], w2s);
            atomicAdd(&grad[kOffB1 + col], b1s);
        }
    }
    if (col_in == 0) {
        atomicAdd(&grad[kOffB2], db2);
        atomicAdd(loss_sum, lsum);
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
    const int64_t tiles = (rows + 31) / 32;
    const int grid = grid_for(tiles, kWaves, 1024);
    if (backward) {
        zero_f32_kernel<<<grid_for(HP_MLP_PARAMS, 256, 64), 256, 0, s>>>(net.grad, HP_MLP_PARAMS);
        zero_f32_kernel<<<1, 64, 0, s>>>(loss_sum, 1);
        mlp_kernel<true><<<grid, kWaves * 64, 0, s>>>(x, y, rows, net.params, net.w_bf16, nullptr, net.grad, loss_sum);
    } else {
        mlp_kernel<false><<<grid, kWaves * 64, 0, s>>>(x, nullptr, rows, net.params, net.w_bf16, q, nullptr, nullptr);
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
