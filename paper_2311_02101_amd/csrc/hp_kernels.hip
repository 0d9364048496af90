// HIP kernels of the block-Gibbs hot path for gfx950 (CDNA4, wave64).
//
// One workgroup advances one chain of one formula through all requested
// sweeps.  The chain's assignment v (one byte per variable) and the hidden
// masks of all its clauses (one byte per clause) stay in LDS for the whole
// launch, the variance EMA stays in registers, so HBM/L2 traffic per sweep is
// only the shared clause table and occurrence lists (the same for every chain
// of a formula, hence L2-resident).
//
// Per sweep (the round of Sec. 3.2 / appendix program, in its order):
//   clause phase  -- for each clause: gather its K inputs from LDS, form the
//                    literal-truth pattern m (bit k set iff literal k is true),
//                    count m != 0, then draw its L hidden units against the
//                    integer thresholds thr[m][l] (eqs. 2, 4, 6) and store the
//                    hidden mask.
//   barrier; the workgroup total gives the satisfied count s; if s > s_max
//                    the current v is copied into best.
//   visible phase -- for each variable: x = sum over its occurrences (c, k),
//                    in ascending (c, k) order, of pol_kc * G[hmask_c][k]
//                    (eq. 7 with d = 0), rho = sigma(x), the variance EMA
//                    (Sec. 3.4) and the draw U < rho.
//   barrier.
#include <hip/hip_runtime.h>

#include "hp_internal.hpp"
#include "philox.hpp"

namespace hp {

// --------------------------------------------------------------------------
// Plan tables (once per plan)
// --------------------------------------------------------------------------
__global__ void tables_kernel(const double *__restrict__ W, const double *__restrict__ b, int K, int L,
                              int T, uint32_t *__restrict__ thr, double *__restrict__ g64,
                              float *__restrict__ g32) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_thr = T * kPatterns * kMaxL;
    const int n_g = T * kHidMasks * kMaxL;
    if (tid < n_thr) {
        const int tau = tid / (kPatterns * kMaxL);
        const int m = (tid / kMaxL) % kPatterns;
        const int l = tid % kMaxL;
        uint32_t out = 0;
        if (l < L && m < (1 << K)) {
            const double *Wt = W + (size_t)tau * K * L;
            double z = b[tau * L + l];
            for (int k = 0; k < K; ++k)
                if ((m >> k) & 1) z += Wt[k * L + l];
            const double p = 1.0 / (1.0 + exp(-z));
            out = (uint32_t)ceil(p * 16777216.0);   // exact scaling by 2^24
        }
        thr[tid] = out;
    }
    if (tid < n_g) {
        const int tau = tid / (kHidMasks * kMaxL);
        const int n = (tid / kMaxL) % kHidMasks;
        const int k = tid % kMaxL;
        double acc = 0.0;
        if (k < K && n < (1 << L)) {
            const double *Wt = W + (size_t)tau * K * L;
            for (int l = 0; l < L; ++l)
                if ((n >> l) & 1) acc += Wt[k * L + l];
        }
        g64[tid] = acc;
        g32[tid] = (float)acc;
    }
}

hipError_t launch_tables(const Plan &p, hipStream_t s) {
    const int n = p.T * kHidMasks * kMaxL;   // >= the threshold table size
    tables_kernel<<<(n + 255) / 256, 256, 0, s>>>(p.d_W, p.d_b, p.K, p.L, p.T, p.tab.thr, p.tab.g64,
                                                  p.tab.g32);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Sweep kernel
// --------------------------------------------------------------------------
__device__ __forceinline__ double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }
__device__ __forceinline__ float sigmoid(float x) { return 1.0f / (1.0f + expf(-x)); }

template <typename Real>
__device__ __forceinline__ Real ema(Real nu, Real rho, Real a) {
    // (1 - a) nu + a rho (1 - rho), evaluated left to right without fusing
#pragma clang fp contract(off)
    const Real one = Real(1);
    return (one - a) * nu + a * rho * (one - rho);
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// VPT > 0: each thread owns VPT groups of 4 consecutive variables and keeps
// their variance EMA in registers.  VPT == 0: any number of groups, EMA read
// and written in global memory every sweep.
template <typename Real, int VPT>
__global__ __launch_bounds__(1024) void sweep_kernel(SweepParams<Real> P) {
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t *s_thr = reinterpret_cast<uint32_t *>(lds);
    Real *s_G = reinterpret_cast<Real *>(lds + kPatterns * kMaxL * 4);
    int *s_cnt = reinterpret_cast<int *>(lds + kPatterns * kMaxL * 4 + kHidMasks * kMaxL * sizeof(Real));
    uint8_t *s_v = lds + P.lds_v_off;
    uint8_t *s_hm = lds + P.lds_hm_off;

    const WorkItem w = P.work[blockIdx.x];
    const FormulaDev fd = P.fd[w.f];
    const int N = fd.n, C = fd.c;
    const int tid = threadIdx.x, NT = blockDim.x;
    const int tau = P.temp_of_chain[w.b];
    const int64_t sbase = fd.var_off * P.B + (int64_t)w.b * N;
    const uint16_t *__restrict__ lits = P.lits + fd.clause_off;
    const uint32_t *__restrict__ cptr = P.csr_ptr + fd.ptr_off;
    const uint32_t *__restrict__ occ = P.occ;
    const Key2 key{P.key0, P.key1 ^ (uint32_t)w.f};
    const bool sample = P.n_sweeps > 0;
    const int64_t S = sample ? P.n_sweeps : 1;
    const uint32_t nbh = (uint32_t)(P.L + 3) >> 2;
    const int K = P.K;
    const int64_t ctot = P.ctot;
    const Real alpha = P.alpha;
    const Real two_m24 = Real(1.0 / 16777216.0);

    for (int i = tid; i < kPatterns * kMaxL; i += NT) s_thr[i] = P.thr[tau * kPatterns * kMaxL + i];
    for (int i = tid; i < kHidMasks * kMaxL; i += NT) s_G[i] = P.G[tau * kHidMasks * kMaxL + i];
    for (int i = tid; i < N; i += NT) s_v[i] = P.v[sbase + i];
    constexpr int VR = VPT > 0 ? VPT : 1;
    Real nu[VR][4];
    if (VPT > 0) {
#pragma unroll
        for (int j = 0; j < VR; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = (tid + j * NT) * 4 + q;
                nu[j][q] = i < N ? P.nu[sbase + i] : Real(0);
            }
    }
    int smax = P.s_max[(int64_t)w.f * P.B + w.b];
    const int64_t t0 = *P.t_ptr;
    __syncthreads();

    for (int64_t s = 0; s < S; ++s) {
        const uint64_t t = (uint64_t)(t0 + s);
        const uint32_t tlo = (uint32_t)t, thi = (uint32_t)(t >> 32);
        // ---- clause phase: gather, count, hidden draw ----
        int cnt = 0;
        for (int c = tid; c < C; c += NT) {
            uint32_t m = 0;
#pragma unroll
            for (int k = 0; k < kMaxK; ++k) {
                if (k < K) {
                    const uint32_t e = lits[(int64_t)k * ctot + c];
                    m |= (uint32_t)(s_v[e & 0x7fffu] ^ (e >> 15)) << k;
                }
            }
            cnt += (m != 0u);
            if (sample) {
                const uint4 t0v = *reinterpret_cast<const uint4 *>(s_thr + m * kMaxL);
                uint4 r = philox4x32_10(make_uint4(tlo, (uint32_t)w.b, kPhaseHidden | ((uint32_t)c * nbh), thi), key);
                uint32_t n = (uint32_t)((r.x >> 8) < t0v.x) | ((uint32_t)((r.y >> 8) < t0v.y) << 1) |
                             ((uint32_t)((r.z >> 8) < t0v.z) << 2) | ((uint32_t)((r.w >> 8) < t0v.w) << 3);
                if (nbh > 1) {
                    const uint4 t1v = *reinterpret_cast<const uint4 *>(s_thr + m * kMaxL + 4);
                    r = philox4x32_10(make_uint4(tlo, (uint32_t)w.b, kPhaseHidden | ((uint32_t)c * nbh + 1u), thi), key);
                    n |= ((uint32_t)((r.x >> 8) < t1v.x) << 4) | ((uint32_t)((r.y >> 8) < t1v.y) << 5) |
                         ((uint32_t)((r.z >> 8) < t1v.z) << 6) | ((uint32_t)((r.w >> 8) < t1v.w) << 7);
                }
                s_hm[c] = (uint8_t)n;
            }
        }
        cnt = wave_sum(cnt);
        if ((tid & (kWave - 1)) == 0) s_cnt[tid / kWave] = cnt;
        __syncthreads();
        int total = 0;
        for (int wv = 0; wv < NT / kWave; ++wv) total += s_cnt[wv];
        const bool improved = total > smax;
        if (improved) smax = total;
        // ---- visible phase: scatter-add (pull), sigmoid, EMA, draw ----
        const int groups = (N + 3) >> 2;
        const int jmax = VPT > 0 ? VPT : (groups + NT - 1) / NT;
#pragma unroll
        for (int j = 0; j < (VPT > 0 ? VPT : 1); ++j) {
          for (int jj = (VPT > 0 ? j : 0); jj < (VPT > 0 ? j + 1 : jmax); ++jj) {
            const int grp = tid + jj * NT;
            if (grp < groups) {
                uint4 r = make_uint4(0, 0, 0, 0);
                if (sample) r = philox4x32_10(make_uint4(tlo, (uint32_t)w.b, kPhaseVisible | (uint32_t)grp, thi), key);
                const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = grp * 4 + q;
                    if (i < N) {
                        const uint8_t old = s_v[i];
                        if (improved) P.best[sbase + i] = old;
                        if (sample) {
                            Real x = Real(0);
                            const uint32_t o1 = cptr[i + 1];
                            for (uint32_t o = cptr[i]; o < o1; ++o) {
                                const uint32_t e = occ[o];
                                const Real g = s_G[(uint32_t)s_hm[e >> 4] * kMaxL + (e & 7u)];
                                x += (e & 8u) ? -g : g;
                            }
                            const Real rho = sigmoid(x);
                            if (VPT > 0) {
                                nu[j][q] = ema(nu[j][q], rho, alpha);
                            } else {
                                P.nu[sbase + i] = ema(P.nu[sbase + i], rho, alpha);
                            }
                            s_v[i] = (Real(rw[q] >> 8) * two_m24) < rho ? 1 : 0;
                        }
                    }
                }
            }
          }
        }
        __syncthreads();
    }
    for (int i = tid; i < N; i += NT) P.v[sbase + i] = s_v[i];
    if (VPT > 0) {
#pragma unroll
        for (int j = 0; j < VR; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = (tid + j * NT) * 4 + q;
                if (i < N) P.nu[sbase + i] = nu[j][q];
            }
    }
    if (tid == 0) P.s_max[(int64_t)w.f * P.B + w.b] = smax;
}

__global__ void advance_t_kernel(int64_t *t, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t[0] += n;
}

template <typename Real, int VPT>
hipError_t launch_one(const Plan &p, const SweepParams<Real> &P, hipStream_t s) {
    auto kern = sweep_kernel<Real, VPT>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)p.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(p.n_work), dim3(p.threads), p.lds_bytes, s, P);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_sweep_t(const Plan &p, const hp_state &st, int64_t n_sweeps, const Real *G,
                          hipStream_t s) {
    SweepParams<Real> P;
    P.fd = p.d_fd;
    P.work = p.d_work;
    P.lits = p.d_lits;
    P.csr_ptr = p.d_csr_ptr;
    P.occ = p.d_occ;
    P.thr = p.tab.thr;
    P.G = G;
    P.temp_of_chain = p.d_temp;
    P.v = st.v;
    P.nu = reinterpret_cast<Real *>(st.nu);
    P.s_max = st.s_max;
    P.best = st.best;
    P.t_ptr = st.t;
    P.ctot = p.total_clauses;
    P.n_sweeps = n_sweeps;
    P.alpha = (Real)p.alpha;
    P.key0 = (uint32_t)(p.seed & 0xffffffffu);
    P.key1 = (uint32_t)(p.seed >> 32);
    P.K = p.K;
    P.L = p.L;
    P.B = p.B;
    P.lds_v_off = p.lds_v_off;
    P.lds_hm_off = p.lds_hm_off;
    hipError_t e;
    switch (p.vpt) {
        case 1: e = launch_one<Real, 1>(p, P, s); break;
        case 2: e = launch_one<Real, 2>(p, P, s); break;
        case 4: e = launch_one<Real, 4>(p, P, s); break;
        case 8: e = launch_one<Real, 8>(p, P, s); break;
        default: e = launch_one<Real, 0>(p, P, s); break;
    }
    if (e != hipSuccess) return e;
    if (n_sweeps > 0) {
        advance_t_kernel<<<1, 64, 0, s>>>(st.t, n_sweeps);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_sweep(const Plan &p, const hp_state &st, int64_t n_sweeps, hipStream_t s) {
    if (p.precision == HP_FP64) return launch_sweep_t<double>(p, st, n_sweeps, p.tab.g64, s);
    return launch_sweep_t<float>(p, st, n_sweeps, p.tab.g32, s);
}

}  // namespace hp
