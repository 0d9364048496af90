// HIP kernels of the block-Gibbs hot path for gfx950 (CDNA4, wave64).
//
// One workgroup advances one chain of one formula through all requested
// sweeps; the chain's state stays on chip for the whole launch (v in LDS, the
// variance EMA in registers), so HBM/L2 traffic per sweep is only the shared
// clause data of the formula (the same for every chain, hence L2-resident).
//
// Two variants of the scatter-add of eq. 7:
//   push (default) -- right after a clause's hidden units are drawn, its
//       contributions pol_kc * G[h-mask][k] are added into per-variable int64
//       fixed-point accumulators in LDS (scale 2^S chosen by the plan so no
//       sum can overflow).  Integer addition is associative, so the result is
//       exact, deterministic and independent of the order of the LDS atomics.
//       Clauses come as 16-byte records sorted by length; the padding copies
//       of a clause's first literal (Sec. 3.3) are merged into one slot.
//   pull -- the hidden masks of all clauses are kept in LDS and every
//       variable sums its contributions over its occurrence list in ascending
//       (clause, position) order in floating point.
//
// Per sweep (the round of Sec. 3.2 / appendix program, in its order), pull:
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

#include <cmath>

namespace hp {

// --------------------------------------------------------------------------
// Plan tables (once per plan)
// --------------------------------------------------------------------------
__device__ double g_entry(const double *__restrict__ Wt, int K, int L, int n, int k) {
    // G[n][k] = sum over the set bits l of n, ascending, of W_c[k,l]
    double acc = 0.0;
    if (k < K && n < (1 << L))
        for (int l = 0; l < L; ++l)
            if ((n >> l) & 1) acc += Wt[k * L + l];
    return acc;
}

__device__ int64_t g_fixed(const double *__restrict__ Wt, int K, int L, int n, int k, int S) {
    return (int64_t)llrint(ldexp(g_entry(Wt, K, L, n, k), S));
}

__global__ void tables_kernel(const double *__restrict__ W, const double *__restrict__ b, int K, int L,
                              int T, int S, uint32_t *__restrict__ thr, double *__restrict__ g64,
                              float *__restrict__ g32, int64_t *__restrict__ gfx,
                              int64_t *__restrict__ gpad) {
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
        const double *Wt = W + (size_t)tau * K * L;
        const double acc = g_entry(Wt, K, L, n, k);
        g64[tid] = acc;
        g32[tid] = (float)acc;
        gfx[tid] = g_fixed(Wt, K, L, n, k, S);
        // gpad[tau][len][n], same flat range: len = tid / 256 % 8, n = tid % 256
        const int len = (tid / kHidMasks) % kMaxL;
        const int n2 = tid % kHidMasks;
        int64_t acc2 = 0;
        if (len >= 1 && len <= K) {
            acc2 = g_fixed(Wt, K, L, n2, 0, S);
            for (int kk = len; kk < K; ++kk) acc2 += g_fixed(Wt, K, L, n2, kk, S);
        }
        gpad[tid] = acc2;
    }
}

hipError_t launch_tables(const Plan &p, hipStream_t s) {
    const int n = p.T * kHidMasks * kMaxL;   // >= the threshold table size
    tables_kernel<<<(n + 255) / 256, 256, 0, s>>>(p.d_W, p.d_b, p.K, p.L, p.T, p.fx_shift, p.tab.thr,
                                                  p.tab.g64, p.tab.g32, p.tab.gfx, p.tab.gpad);
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

size_t lds_bytes_pull(int max_n, int max_c, size_t real_bytes, int32_t *v_off, int32_t *hm_off) {
    size_t off = (size_t)kPatterns * kMaxL * 4 + (size_t)kHidMasks * kMaxL * real_bytes + 64 * 4;
    *v_off = (int32_t)off;
    off += ((size_t)max_n + 15) / 16 * 16;
    *hm_off = (int32_t)off;
    off += ((size_t)max_c + 15) / 16 * 16;
    return off;
}

// push LDS layout: thr (4 KB) | gfx (16 KB) | gpad (16 KB) | counts | x (8 B/var) | v (1 B/var)
constexpr int kPushGfxOff = kPatterns * kMaxL * 4;
constexpr int kPushGpadOff = kPushGfxOff + kHidMasks * kMaxL * 8;
constexpr int kPushCntOff = kPushGpadOff + kMaxL * kHidMasks * 8;
constexpr int kPushXOff = kPushCntOff + 64 * 4;

size_t lds_bytes_push(int max_n, int32_t *v_off, int32_t *x_off) {
    size_t off = kPushXOff;
    *x_off = (int32_t)off;
    off += (size_t)max_n * 8;
    *v_off = (int32_t)off;
    off += ((size_t)max_n + 15) / 16 * 16;
    return off;
}

// VPT > 0: each thread owns VPT groups of 4 consecutive variables and keeps
// their variance EMA in registers.  VPT == 0: any number of groups, EMA read
// and written in global memory every sweep.
template <typename Real, int VPT>
__global__ __launch_bounds__(1024) void sweep_pull_kernel(SweepParams<Real> P) {
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

// literal truth of a 16-bit clause slot: v[index] xor negated
__device__ __forceinline__ uint32_t lit_of(const uint8_t *s_v, uint32_t e) {
    return (uint32_t)s_v[e & 0x7fffu] ^ (e >> 15);
}

__device__ __forceinline__ void push_add(int64_t *s_x, uint32_t e, int64_t g) {
    atomicAdd(reinterpret_cast<unsigned long long *>(&s_x[e & 0x7fffu]),
              (unsigned long long)((e >> 15) ? -g : g));
}

template <typename Real, int VPT>
__global__ __launch_bounds__(1024) void sweep_push_kernel(SweepParams<Real> P) {
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t *s_thr = reinterpret_cast<uint32_t *>(lds);
    int64_t *s_gfx = reinterpret_cast<int64_t *>(lds + kPushGfxOff);
    int64_t *s_gpad = reinterpret_cast<int64_t *>(lds + kPushGpadOff);
    int *s_cnt = reinterpret_cast<int *>(lds + kPushCntOff);
    int64_t *s_x = reinterpret_cast<int64_t *>(lds + P.lds_x_off);
    uint8_t *s_v = lds + P.lds_v_off;

    const WorkItem w = P.work[blockIdx.x];
    const FormulaDev fd = P.fd[w.f];
    const int N = fd.n, C = fd.c;
    const int tid = threadIdx.x, NT = blockDim.x;
    const int tau = P.temp_of_chain[w.b];
    const int64_t sbase = fd.var_off * P.B + (int64_t)w.b * N;
    const uint4 *__restrict__ rec = P.rec + fd.clause_off;
    const uint32_t *__restrict__ orig = P.orig + fd.clause_off;
    const Key2 key{P.key0, P.key1 ^ (uint32_t)w.f};
    const bool sample = P.n_sweeps > 0;
    const int64_t S = sample ? P.n_sweeps : 1;
    const uint32_t nbh = (uint32_t)(P.L + 3) >> 2;
    const uint32_t full = (1u << P.K) - 1u;
    const Real alpha = P.alpha;
    const double fx_scale = P.fx_scale;
    const Real two_m24 = Real(1.0 / 16777216.0);

    for (int i = tid; i < kPatterns * kMaxL; i += NT) s_thr[i] = P.thr[tau * kPatterns * kMaxL + i];
    for (int i = tid; i < kHidMasks * kMaxL; i += NT) {
        s_gfx[i] = P.gfx[tau * kHidMasks * kMaxL + i];
        s_gpad[i] = P.gpad[tau * kHidMasks * kMaxL + i];
    }
    for (int i = tid; i < N; i += NT) {
        s_v[i] = P.v[sbase + i];
        s_x[i] = 0;
    }
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
        // ---- clause phase: gather, count, hidden draw, scatter into x ----
        int cnt = 0;
        uint4 r_next = make_uint4(0, 0, 0, 0);
        uint32_t o_next = 0;
        if (tid < C) {
            r_next = rec[tid];
            o_next = orig[tid];
        }
        for (int c = tid; c < C; c += NT) {
            const uint4 r = r_next;
            const uint32_t oc = o_next;
            if (c + NT < C) {           // prefetch the next record
                r_next = rec[c + NT];
                o_next = orig[c + NT];
            }
            const uint32_t len = r.w >> 16;
            const uint32_t e0 = r.x & 0xffffu, e1 = r.x >> 16, e2 = r.y & 0xffffu, e3 = r.y >> 16;
            const uint32_t e4 = r.z & 0xffffu, e5 = r.z >> 16, e6 = r.w & 0xffffu;
            const uint32_t l0 = lit_of(s_v, e0);
            uint32_t m = l0;
            if (len > 1) m |= lit_of(s_v, e1) << 1;
            if (len > 2) m |= lit_of(s_v, e2) << 2;
            if (len > 3) m |= lit_of(s_v, e3) << 3;
            if (len > 4) m |= lit_of(s_v, e4) << 4;
            if (len > 5) m |= lit_of(s_v, e5) << 5;
            if (len > 6) m |= lit_of(s_v, e6) << 6;
            m |= l0 ? (full & ~((1u << len) - 1u)) : 0u;   // padding copies of literal 0
            cnt += (m != 0u);
            if (sample) {
                const uint4 ta = *reinterpret_cast<const uint4 *>(s_thr + m * kMaxL);
                uint4 ra = philox4x32_10(make_uint4(tlo, (uint32_t)w.b, kPhaseHidden | (oc * nbh), thi), key);
                uint32_t n = (uint32_t)((ra.x >> 8) < ta.x) | ((uint32_t)((ra.y >> 8) < ta.y) << 1) |
                             ((uint32_t)((ra.z >> 8) < ta.z) << 2) | ((uint32_t)((ra.w >> 8) < ta.w) << 3);
                if (nbh > 1) {
                    const uint4 tb = *reinterpret_cast<const uint4 *>(s_thr + m * kMaxL + 4);
                    const uint4 rb = philox4x32_10(make_uint4(tlo, (uint32_t)w.b, kPhaseHidden | (oc * nbh + 1u), thi), key);
                    n |= ((uint32_t)((rb.x >> 8) < tb.x) << 4) | ((uint32_t)((rb.y >> 8) < tb.y) << 5) |
                         ((uint32_t)((rb.z >> 8) < tb.z) << 6) | ((uint32_t)((rb.w >> 8) < tb.w) << 7);
                }
                push_add(s_x, e0, s_gpad[len * kHidMasks + n]);
                const int64_t *gr = s_gfx + n * kMaxL;
                if (len > 1) push_add(s_x, e1, gr[1]);
                if (len > 2) push_add(s_x, e2, gr[2]);
                if (len > 3) push_add(s_x, e3, gr[3]);
                if (len > 4) push_add(s_x, e4, gr[4]);
                if (len > 5) push_add(s_x, e5, gr[5]);
                if (len > 6) push_add(s_x, e6, gr[6]);
            }
        }
        cnt = wave_sum(cnt);
        if ((tid & (kWave - 1)) == 0) s_cnt[tid / kWave] = cnt;
        __syncthreads();
        int total = 0;
        for (int wv = 0; wv < NT / kWave; ++wv) total += s_cnt[wv];
        const bool improved = total > smax;
        if (improved) smax = total;
        // ---- visible phase: sigmoid of the accumulated logit, EMA, draw ----
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
                            const int64_t xi = s_x[i];
                            s_x[i] = 0;
                            const Real x = (Real)((double)xi * fx_scale);
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
hipError_t launch_one(bool push, int n_items, size_t lds, int threads, SweepParams<Real> P, hipStream_t s) {
    auto kern = push ? sweep_push_kernel<Real, VPT> : sweep_pull_kernel<Real, VPT>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(threads), lds, s, P);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_variant(bool push, int vpt, int n_items, size_t lds, int threads,
                          const SweepParams<Real> &P, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    switch (vpt) {
        case 1: return launch_one<Real, 1>(push, n_items, lds, threads, P, s);
        case 2: return launch_one<Real, 2>(push, n_items, lds, threads, P, s);
        default: return launch_one<Real, 0>(push, n_items, lds, threads, P, s);
    }
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
    P.rec = p.d_rec;
    P.orig = p.d_orig;
    P.gfx = p.tab.gfx;
    P.gpad = p.tab.gpad;
    P.fx_scale = std::ldexp(1.0, -p.fx_shift);
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
    // push launch over work items [0, n_push)
    P.lds_v_off = p.push_v_off;
    P.lds_x_off = p.push_x_off;
    P.lds_hm_off = 0;
    hipError_t e = launch_variant<Real>(true, p.vpt_push, p.n_push, p.lds_push, p.threads, P, s);
    if (e != hipSuccess) return e;
    // pull launch over work items [n_push, n_work)
    P.work = p.d_work + p.n_push;
    P.lds_v_off = p.pull_v_off;
    P.lds_hm_off = p.pull_hm_off;
    P.lds_x_off = 0;
    e = launch_variant<Real>(false, p.vpt_pull, p.n_work - p.n_push, p.lds_pull, p.threads, P, s);
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
