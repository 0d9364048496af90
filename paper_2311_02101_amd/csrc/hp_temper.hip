// Replica exchange across the temperatures (the ensemble of free-energy
// targets).  Chain b of formula f samples the formula-RBM of temperature tau,
// whose visible marginal is p_tau(v) ~ exp(-F_tau(v)), F_tau the formula free
// energy (eq. 5): the sum over clauses of the clause free energy (eq. 1) of
// the clause's literal values (eq. 4).  A round pairs, in every formula, the
// k-th chain (by index) at tau with the k-th chain at tau + 1 for the pairs
// (tau, tau+1) of one parity and exchanges their temperatures with
// probability min(1, exp(D)),
//     D = F_tau(v_a) + F_tau+1(v_b) - F_tau(v_b) - F_tau+1(v_a),
// the draw U = (w >> 8) 2^-24 from word 0 of Philox4x32-10 at counter
// (t mod 2^32, a, 2^31 - 1, t div 2^32) with the sweep generator's key.
// In the size-clustered model every clause contributes the free energy of
// its own group's RBM.
#include <hip/hip_runtime.h>

#include "hp_internal.hpp"
#include "philox.hpp"

namespace hp {

constexpr int kFeThreads = 256;
constexpr uint32_t kSwapBlock = 0x7fffffffu;

__device__ __forceinline__ double softplus(double z) { return z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z)); }

// fe[tau][m] = -sum_l softplus(b_l + sum_k bit_k(m) W_kl) for patterns m < 2^K
__global__ void fe_table_kernel(const double *__restrict__ W, const double *__restrict__ b, int K, int L, int T,
                                double *__restrict__ fe) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T * kPatterns) return;
    const int tau = i / kPatterns, m = i % kPatterns;
    double f = 0.0;
    if (m < (1 << K)) {
        const double *Wt = W + (size_t)tau * K * L;
        for (int l = 0; l < L; ++l) {
            double z = b[tau * L + l];
            for (int k = 0; k < K; ++k)
                if ((m >> k) & 1) z += Wt[k * L + l];
            f -= softplus(z);
        }
    }
    fe[i] = f;
}

// Size-clustered model: fe[tau][r] over the 248 pattern rows of the five
// groups (group K at row 2^K - 8), each with its own RBM.
__global__ void fe_table_clust_kernel(ClustRbm R, int T, double *__restrict__ fe) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T * kClustThrRows) return;
    const int tau = i / kClustThrRows, row = i % kClustThrRows;
    const int K = 31 - __clz(row + 8), L = clust_hidden(K), m = row - ((1 << K) - 8);
    double f = 0.0;
    if (R.W[K - 3]) {
        const double *Wt = R.W[K - 3] + (size_t)tau * K * L;
        for (int l = 0; l < L; ++l) {
            double z = R.b[K - 3][tau * L + l];
            for (int k = 0; k < K; ++k)
                if ((m >> k) & 1) z += Wt[k * L + l];
            f -= softplus(z);
        }
    }
    fe[i] = f;
}

// F_tau(v) of every (formula, chain) for every temperature: [F][B][T].
// kClust: a clause of length len reads row 2^K - 8 + m of the clustered
// table, K = max(len, 3), m its pattern padded to K inputs.
template <bool kClust>
__global__ __launch_bounds__(kFeThreads) void free_energy_kernel(const FormulaDev *__restrict__ fd,
                                                                 const WorkItem *__restrict__ work,
                                                                 const uint4 *__restrict__ rec, int B, int T,
                                                                 uint32_t full, const uint8_t *__restrict__ v,
                                                                 const double *__restrict__ fe,
                                                                 double *__restrict__ out) {
    __shared__ double s_part[kFeThreads / kWave][kMaxTemperTemps];
    const WorkItem w = work[blockIdx.x];
    const FormulaDev f = fd[w.f];
    const uint8_t *vb = v + f.var_off * B + (int64_t)w.b * f.n;
    const uint4 *r = rec + f.clause_off;
    double acc[kMaxTemperTemps];
    for (int t = 0; t < kMaxTemperTemps; ++t) acc[t] = 0.0;
    for (int c = threadIdx.x; c < f.c; c += blockDim.x) {
        const uint4 q = r[c];
        const uint32_t len = rec_len(q.w), negm = rec_negm(q.w);
        const uint32_t e[7] = {q.x & 0xffffu, q.x >> 16, q.y & 0xffffu, q.y >> 16,
                               q.z & 0xffffu, q.z >> 16, q.w & 0xffffu};
        uint32_t m = 0;
        for (uint32_t k = 0; k < len; ++k) m |= (uint32_t)(vb[e[k] & 0x7fffu] & 1u) << k;
        const uint32_t lenmask = (1u << len) - 1u;
        m = (m ^ negm) & lenmask;
        if (kClust) {
            const uint32_t Kc = len < 3u ? 3u : len;
            m |= (m & 1u) ? (((1u << Kc) - 1u) & ~lenmask) : 0u;
            const uint32_t row = (1u << Kc) - 8u + m;
            for (int t = 0; t < T; ++t) acc[t] += fe[t * kClustThrRows + row];
        } else {
            m |= (m & 1u) ? (full & ~lenmask) : 0u;          // padding copies of literal 0
            for (int t = 0; t < T; ++t) acc[t] += fe[t * kPatterns + m];
        }
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int t = 0; t < T; ++t) {
        double x = acc[t];
        for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
        if (lane == 0) s_part[wave][t] = x;
    }
    __syncthreads();
    if ((int)threadIdx.x < T) {
        double x = 0.0;
        for (int i = 0; i < (int)blockDim.x / kWave; ++i) x += s_part[i][threadIdx.x];
        out[(size_t)blockIdx.x * T + threadIdx.x] = x;
    }
}

// one swap round per formula (a single thread walks the pairs in order)
__global__ void swap_kernel(const int32_t *__restrict__ temp_old, int32_t *__restrict__ temp,
                            const double *__restrict__ F, int B, int T, int parity, const int64_t *__restrict__ t_ptr,
                            uint32_t key0, uint32_t key1) {
    if (threadIdx.x != 0) return;
    const int f = blockIdx.x;
    const uint64_t t = (uint64_t)*t_ptr;
    const int32_t *to = temp_old + (size_t)f * B;
    int32_t *tn = temp + (size_t)f * B;
    const double *Ff = F + (size_t)f * B * T;
    const Key2 key{key0, key1 ^ (uint32_t)f};
    for (int tau = parity; tau + 1 < T; tau += 2) {
        int a = 0, c = 0;
        for (;;) {
            while (a < B && to[a] != tau) ++a;
            while (c < B && to[c] != tau + 1) ++c;
            if (a >= B || c >= B) break;
            const double D = Ff[(size_t)a * T + tau] + Ff[(size_t)c * T + tau + 1] - Ff[(size_t)c * T + tau] -
                             Ff[(size_t)a * T + tau + 1];
            const uint4 rw = philox4x32_10_lane_key(make_uint4((uint32_t)t, (uint32_t)a, kSwapBlock,
                                                               (uint32_t)(t >> 32)), key);
            const double u = (double)(rw.x >> 8) * (1.0 / 16777216.0);
            if (u < exp(D < 0.0 ? D : 0.0)) {
                tn[a] = tau + 1;
                tn[c] = tau;
            }
            ++a;
            ++c;
        }
    }
}

hipError_t launch_temper(Plan &p, const hp_state &st, int parity, hipStream_t s) {
    const size_t items = (size_t)p.F * p.B;
    const int rows = p.clust ? kClustThrRows : kPatterns;
    if (!p.d_fe) {
        hipError_t e = hipMalloc((void **)&p.d_fe, (size_t)p.T * rows * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void **)&p.d_fe_chain, items * p.T * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void **)&p.d_temp_old, items * sizeof(int32_t));
        if (e != hipSuccess) return e;
        if (p.clust)
            fe_table_clust_kernel<<<(p.T * rows + 255) / 256, 256, 0, s>>>(p.crbm, p.T, p.d_fe);
        else
            fe_table_kernel<<<(p.T * rows + 255) / 256, 256, 0, s>>>(p.d_W, p.d_b, p.K, p.L, p.T, p.d_fe);
    }
    hipError_t e = hipMemcpyAsync(p.d_temp_old, p.d_temp, items * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    if (p.clust)
        free_energy_kernel<true><<<(unsigned)items, kFeThreads, 0, s>>>(p.d_fd, p.d_work_fb, p.d_rec, p.B, p.T, 0u,
                                                                        st.v, p.d_fe, p.d_fe_chain);
    else
        free_energy_kernel<false><<<(unsigned)items, kFeThreads, 0, s>>>(p.d_fd, p.d_work_fb, p.d_rec, p.B, p.T,
                                                                         (1u << p.K) - 1u, st.v, p.d_fe, p.d_fe_chain);
    swap_kernel<<<p.F, 64, 0, s>>>(p.d_temp_old, p.d_temp, p.d_fe_chain, p.B, p.T, parity, st.t,
                                   (uint32_t)(p.seed & 0xffffffffu), (uint32_t)(p.seed >> 32));
    return hipGetLastError();
}

}  // namespace hp
