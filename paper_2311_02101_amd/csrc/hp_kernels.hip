// HIP kernels of the block-Gibbs hot path for gfx950 (CDNA4, wave64).
//
// One workgroup advances one chain of one formula through all requested
// sweeps; the chain's state stays on chip for the whole launch (v in LDS, the
// variance EMA in registers), so HBM/L2 traffic per sweep is only the shared
// clause data of the formula and, in the wide and mid table layouts, the
// contribution rows of the chain's temperature (the same for every chain of
// the formula, hence L2-resident).
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

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

namespace hp {

// --------------------------------------------------------------------------
// Plan tables (once per plan)
// --------------------------------------------------------------------------
__device__ double g_entry(const double *__restrict__ Wt, int K, int L, int n, int k) {
    // G[n][k] = sum over the set bits l < L of n, ascending, of W_c[k,l]; the
    // bits of n at and above L are ignored, so rows n >= 2^L repeat row
    // n mod 2^L (the push kernels index them with undrawn high units)
    double acc = 0.0;
    if (k < K)
        for (int l = 0; l < L; ++l)
            if ((n >> l) & 1) acc += Wt[k * L + l];
    return acc;
}

__device__ int64_t g_fixed(const double *__restrict__ Wt, int K, int L, int n, int k, int S) {
    return (int64_t)llrint(ldexp(g_entry(Wt, K, L, n, k), S));
}

__global__ void tables_kernel(const double *__restrict__ W, const double *__restrict__ b, int K, int L,
                              int T, int S, uint32_t *__restrict__ thr, double *__restrict__ g64,
                              float *__restrict__ g32, int64_t *__restrict__ gtab, int32_t *__restrict__ flag) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_thr = T * kPatterns * kMaxL;
    const int n_g = T * kHidMasks * kMaxL;
    const int n_tab = T * kHidMasks * kRowWords;
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
            // c = ceil(2^24 p) (exact scaling); U < p  <=>  (word >> 8) < c
            // <=>  word <= 256 c - 1, which fits 32 bits for 1 <= c <= 2^24
            const uint32_t c = (uint32_t)ceil(p * 16777216.0);
            if (c == 0u) *flag = 1;               // p underflowed to 0: not representable
            out = c * 256u - 1u;
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
    }
    if (tid < n_tab) {
        // gtab[tau][n][j]: j < 8 the fixed-point G[n][j]; j = 8 + len the
        // merged contribution of a clause of len literals to its first one
        const int tau = tid / (kHidMasks * kRowWords);
        const int n = (tid / kRowWords) % kHidMasks;
        const int j = tid % kRowWords;
        const double *Wt = W + (size_t)tau * K * L;
        int64_t out = 0;
        if (j < kMaxL) {
            out = g_fixed(Wt, K, L, n, j, S);
        } else if (j - kMaxL >= 1 && j - kMaxL <= K) {
            out = g_fixed(Wt, K, L, n, 0, S);
            for (int kk = j - kMaxL; kk < K; ++kk) out += g_fixed(Wt, K, L, n, kk, S);
        }
        gtab[tid] = out;
    }
}

// Size-clustered tables: one thread per entry of the largest per-temperature
// table (gfx, 488 x 8); the row offsets are the closed forms of the layout.
__global__ void clust_tables_kernel(ClustRbm R, int T, int S, uint32_t *__restrict__ thr,
                                    int64_t *__restrict__ gfx, int64_t *__restrict__ gpad,
                                    int32_t *__restrict__ flag) {
    constexpr int per = kClustGfxRows * kMaxL;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= T * per) return;
    const int tau = tid / per, r = tid % per;
    if (r < kClustThrRows * kMaxL) {
        const int row = r / kMaxL, l = r % kMaxL;
        const int K = 31 - __clz(row + 8);                 // row in [2^K - 8, 2^(K+1) - 8)
        const int L = clust_hidden(K), m = row - ((1 << K) - 8);
        uint32_t out = 0;
        if (l < L && R.W[K - 3]) {
            const double *Wt = R.W[K - 3] + (size_t)tau * K * L;
            double z = R.b[K - 3][tau * L + l];
            for (int k = 0; k < K; ++k)
                if ((m >> k) & 1) z += Wt[k * L + l];
            const double pr = 1.0 / (1.0 + exp(-z));
            const uint32_t c = (uint32_t)ceil(pr * 16777216.0);
            if (c == 0u) *flag = 1;
            out = c * 256u - 1u;
        }
        thr[(size_t)tau * kClustThrRows * kMaxL + r] = out;
    }
    {
        const int row = r / kMaxL, k = r % kMaxL;
        const int K = row < 8 ? 3 : 30 - __clz(row + 24);  // row in [2^(K+1) - 24, 2^(K+2) - 24)
        const int L = clust_hidden(K), n = row - (K == 3 ? 0 : (2 << K) - 24);
        gfx[(size_t)tau * per + r] = R.W[K - 3] ? g_fixed(R.W[K - 3] + (size_t)tau * K * L, K, L, n, k, S) : 0;
    }
    if (r < kClustGpad) {
        const int len = r < 24 ? r / 8 + 1 : 30 - __clz(r + 8);
        const int K = len < 3 ? 3 : len, L = clust_hidden(K);
        const int n = r - (len <= 3 ? 8 * (len - 1) : (2 << len) - 8);
        int64_t acc = 0;
        if (R.W[K - 3]) {
            const double *Wt = R.W[K - 3] + (size_t)tau * K * L;
            acc = g_fixed(Wt, K, L, n, 0, S);
            for (int kk = len; kk < K; ++kk) acc += g_fixed(Wt, K, L, n, kk, S);
        }
        gpad[(size_t)tau * kClustGpad + r] = acc;
    }
}

hipError_t launch_tables(const Plan &p, hipStream_t s) {
    if (p.clust) {
        const int n = p.T * kClustGfxRows * kMaxL;
        clust_tables_kernel<<<(n + 255) / 256, 256, 0, s>>>(p.crbm, p.T, p.fx_shift, p.tab.thr, p.tab.gfx,
                                                            p.tab.gpad, p.d_tabflag);
        return hipGetLastError();
    }
    const int n = p.T * kHidMasks * kRowWords;   // the largest of the three tables
    tables_kernel<<<(n + 255) / 256, 256, 0, s>>>(p.d_W, p.d_b, p.K, p.L, p.T, p.fx_shift, p.tab.thr,
                                                  p.tab.g64, p.tab.g32, p.tab.gfx, p.d_tabflag);
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

// push LDS layout: thr (8 KB) | table rows (32 KB) | counts | v (1 B/var) | x (8 B/var)
// The push kernels' threshold rows are indexed by clause length and the
// pattern of the clause's own literals: row 2^len - 2 + m for len = 1..7
// holds the row of the padded pattern (m with positions >= len copying bit
// 0), so the clause loop never builds the padding bits.
// The contribution table of the padded model has one 128-byte row per
// hidden mask n: words 0..7 the slot contributions, word 8 + len the merged
// contribution of a clause of len literals to its first one, so one offset
// n * 128 addresses both of a clause's reads.
constexpr int kPushTabOff = kThrRows * kMaxL * 4;
constexpr int kPushCntOff = kPushTabOff + kHidMasks * kRowWords * 8;
constexpr int kPushVOff = kPushCntOff + 64 * 4;

// wide layout (table rows read from global memory): thr | counts | v | x
constexpr int kWideCntOff = kThrRows * kMaxL * 4;
constexpr int kWideVOff = kWideCntOff + 64 * 4;

// middle layout (only the merged padding words, one read per clause, from
// global memory): thr | slot contributions (rows of 8) | counts | v | x
constexpr int kMidGfxOff = kThrRows * kMaxL * 4;
constexpr int kMidCntOff = kMidGfxOff + kHidMasks * kMaxL * 8;
constexpr int kMidVOff = kMidCntOff + 64 * 4;

// size-clustered layout: thr (248 rows) | gfx (488 rows) | gpad (504) | counts | v | x
constexpr int kClustGfxOff = kClustThrRows * kMaxL * 4;
constexpr int kClustGpadOff = kClustGfxOff + kClustGfxRows * kMaxL * 8;
constexpr int kClustCntOff = kClustGpadOff + kClustGpad * 8;
constexpr int kClustVOff = kClustCntOff + 64 * 4;

// v sits at a fixed offset (below 64 KB), so a gather is one LDS read with
// the offset in the instruction; x follows, 16-byte aligned
static size_t lds_tail(size_t off, int max_n, int32_t *v_off, int32_t *x_off) {
    *v_off = (int32_t)off;
    off += ((size_t)max_n + 15) / 16 * 16;
    *x_off = (int32_t)off;
    off += (size_t)max_n * 8;
    return off;
}

size_t lds_bytes_push(int max_n, int kind, int32_t *v_off, int32_t *x_off) {
    return lds_tail(kind == kBucketWide ? kWideVOff : kind == kBucketMid ? kMidVOff : kPushVOff, max_n, v_off, x_off);
}

size_t lds_bytes_clust(int max_n, int32_t *v_off, int32_t *x_off) {
    return lds_tail(kClustVOff, max_n, v_off, x_off);
}

// Hidden draw of one clause: L Bernoulli bits against the pre-shifted
// thresholds row[l] = 256 ceil(2^24 p_l) - 1 of its literal pattern, bit l
// set iff word_l <= row[l] (i.e. U < p_l).  Units of the first Philox block
// go to bits 0..3, of the second block (L > 4) to bits 4..7; bits >= L are
// left to the caller to mask.  The bits are shifted in one unit at a time,
// from the highest unit down so that unit l lands on bit l: the compare's
// lane mask is the carry-in of an add that doubles the mask, two VALU
// instructions per unit (a compare, a select and part of an OR in the plain
// C form).
__device__ __forceinline__ uint32_t draw_first(uint32_t w, uint32_t t) {
    uint32_t m;
    asm("v_cmp_le_u32 vcc, %1, %2\n\tv_cndmask_b32_e64 %0, 0, 1, vcc" : "=v"(m) : "v"(w), "v"(t) : "vcc");
    return m;
}
__device__ __forceinline__ uint32_t draw_next(uint32_t m, uint32_t w, uint32_t t) {
    asm("v_cmp_le_u32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, %0, %0, vcc" : "+v"(m) : "v"(w), "v"(t) : "vcc");
    return m;
}

// NB: Philox blocks per clause, 1 (L <= 4) or 2 (L <= 8); 0 = read nbh at run time
template <int NB = 0>
__device__ __forceinline__ uint32_t hidden_mask(const uint32_t *row, uint32_t blk, const PhiloxSweep &u, Key2 key,
                                                uint32_t nbh) {
    const uint4 ta = *reinterpret_cast<const uint4 *>(row);
    if (NB == 2 || (NB == 0 && nbh > 1)) {
        // both blocks in one pass (interleaved rounds, one key schedule)
        const uint4 tb = *reinterpret_cast<const uint4 *>(row + 4);
        uint4 r[2];
        philox_sweep_pair(r, kPhaseHidden | blk, u, key);     // blocks blk, blk + 1 (blk even, < 2^31)
        uint32_t m = draw_first(r[1].w, tb.w);
        m = draw_next(m, r[1].z, tb.z);
        m = draw_next(m, r[1].y, tb.y);
        m = draw_next(m, r[1].x, tb.x);
        m = draw_next(m, r[0].w, ta.w);
        m = draw_next(m, r[0].z, ta.z);
        m = draw_next(m, r[0].y, ta.y);
        return draw_next(m, r[0].x, ta.x);
    }
    const uint4 r = philox_sweep(kPhaseHidden | blk, u, key);
    uint32_t m = draw_first(r.w, ta.w);
    m = draw_next(m, r.z, ta.z);
    m = draw_next(m, r.y, ta.y);
    return draw_next(m, r.x, ta.x);
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
    const int tau = P.temp_of_chain[(int64_t)w.f * P.B + w.b];
    const int64_t sbase = fd.var_off * P.B + (int64_t)w.b * N;
    const uint16_t *__restrict__ lits = P.lits + fd.clause_off;
    const uint32_t *__restrict__ cptr = P.csr_ptr + fd.ptr_off;
    const uint32_t *__restrict__ occ = P.occ;
    const Key2 key{P.key0, P.key1 ^ (uint32_t)w.f};
    const bool sample = P.n_sweeps > 0;
    const int64_t S = sample ? P.n_sweeps : 1;
    const uint32_t nbh = (uint32_t)(P.L + 3) >> 2;
    const uint32_t lmask = (1u << P.L) - 1u;
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
        const PhiloxSweep ps = philox_sweep_consts((uint32_t)t, (uint32_t)w.b, (uint32_t)(t >> 32), key);
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
                uint32_t n = hidden_mask(s_thr + m * kMaxL, (uint32_t)c * nbh, ps, key, nbh) & lmask;
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
                if (sample) r = philox_sweep(kPhaseVisible | (uint32_t)grp, ps, key);
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

// Add pol * g to the accumulator of variable i; sm = 0 for a positive slot,
// all ones for a negated one, which adds ~g = -g - 1.  The missing +1 of every
// negated slot of a variable is a constant of the formula (negcnt) that seeds
// the accumulator.
__device__ __forceinline__ void push_add(int64_t *s_x, uint32_t i, uint32_t sm, int64_t g) {
    const uint64_t u = (uint64_t)g;
    const uint64_t gx = ((uint64_t)((uint32_t)(u >> 32) ^ sm) << 32) | (uint64_t)((uint32_t)u ^ sm);
    atomicAdd(reinterpret_cast<unsigned long long *>(&s_x[i]), (unsigned long long)gx);
}

// the same for a 16-bit clause slot e (variable in bits 0..14, negation in 15)
__device__ __forceinline__ void push_add(int64_t *s_x, uint32_t e, int64_t g) {
    push_add(s_x, e & 0x7fffu, (uint32_t)((int32_t)(e << 16) >> 31), g);
}

// variable and negation mask of slot k of a record (two 16-bit slots a word)
template <int k>
__device__ __forceinline__ uint32_t slot_var(const uint4 &r) {
    const uint32_t w = k < 2 ? r.x : k < 4 ? r.y : k < 6 ? r.z : r.w;
    return (k & 1) ? __builtin_amdgcn_ubfe(w, 16, 15) : (w & 0x7fffu);
}
template <int k>
__device__ __forceinline__ uint32_t slot_neg(const uint4 &r) {
    const uint32_t w = k < 2 ? r.x : k < 4 ? r.y : k < 6 ? r.z : r.w;
    return (uint32_t)__builtin_amdgcn_sbfe((int)w, (k & 1) ? 31 : 15, 1);
}

// The gathers and the table reads go through pointers made from constant
// byte offsets in the workgroup's dynamic LDS (the sweep kernels have no
// static LDS, so it starts at 0): the offset folds into the read instruction
// instead of an add of the array's base address per access.  (The same form
// for the accumulators measured slower in the split launch.)
__device__ __forceinline__ unsigned char *lds_at(int off) {
    return (unsigned char *)(__attribute__((address_space(3))) unsigned char *)(size_t)off;
}

// the third descriptor word of a raw (untyped) buffer on gfx9-family GPUs
constexpr int kRawBufferWord3 = 0x00020000;

// Views of a push layout: LDS regions, plus a buffer descriptor over the
// global table rows of the chain's temperature (mid and wide layouts).
// gfx: the table rows (push layout, rows of 16 words), the slot
// contributions (mid layout, rows of 8) or the size-clustered model's
// contribution rows; gpad: the size-clustered model's merged paddings.
struct PushLds {
    uint32_t *thr;
    int64_t *gfx;
    int64_t *gpad;
    int *cnt;
    int64_t *x;
    uint8_t *v;
    __amdgpu_buffer_rsrc_t grs;
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t table_rows(const int64_t *gtab, int tau) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<int64_t *>(gtab + (size_t)tau * kHidMasks * kRowWords),
                                             (short)0, kHidMasks * kRowWords * 8, kRawBufferWord3);
}

// an empty descriptor (every load through it returns zeros) for the layouts
// that read no table from global memory
__device__ __forceinline__ __amdgpu_buffer_rsrc_t no_rows() {
    return __builtin_amdgcn_make_buffer_rsrc(nullptr, (short)0, 0, kRawBufferWord3);
}

__device__ __forceinline__ PushLds push_lds(unsigned char *lds, int x_off) {
    return PushLds{reinterpret_cast<uint32_t *>(lds_at(0)), reinterpret_cast<int64_t *>(lds_at(kPushTabOff)),
                   nullptr, reinterpret_cast<int *>(lds + kPushCntOff), reinterpret_cast<int64_t *>(lds + x_off),
                   lds_at(kPushVOff), no_rows()};
}

// wide variant: the table rows of temperature tau stay in global memory
__device__ __forceinline__ PushLds push_lds_wide(unsigned char *lds, int x_off, const int64_t *gtab, int tau) {
    return PushLds{reinterpret_cast<uint32_t *>(lds), nullptr, nullptr, reinterpret_cast<int *>(lds + kWideCntOff),
                   reinterpret_cast<int64_t *>(lds + x_off), lds_at(kWideVOff), table_rows(gtab, tau)};
}

// middle variant: the merged paddings of temperature tau stay in global memory
__device__ __forceinline__ PushLds push_lds_mid(unsigned char *lds, int x_off, const int64_t *gtab, int tau) {
    return PushLds{reinterpret_cast<uint32_t *>(lds_at(0)), reinterpret_cast<int64_t *>(lds_at(kMidGfxOff)),
                   nullptr, reinterpret_cast<int *>(lds + kMidCntOff), reinterpret_cast<int64_t *>(lds + x_off),
                   lds_at(kMidVOff), table_rows(gtab, tau)};
}

template <int kTab>
__device__ __forceinline__ PushLds push_lds_for(unsigned char *lds, int x_off, const int64_t *gtab, int tau) {
    if (kTab == kBucketWide) return push_lds_wide(lds, x_off, gtab, tau);
    if (kTab == kBucketMid) return push_lds_mid(lds, x_off, gtab, tau);
    return push_lds(lds, x_off);
}

__device__ __forceinline__ PushLds push_lds_clust(unsigned char *lds, int x_off) {
    return PushLds{reinterpret_cast<uint32_t *>(lds_at(0)), reinterpret_cast<int64_t *>(lds_at(kClustGfxOff)),
                   reinterpret_cast<int64_t *>(lds_at(kClustGpadOff)), reinterpret_cast<int *>(lds + kClustCntOff),
                   reinterpret_cast<int64_t *>(lds + x_off), lds_at(kClustVOff), no_rows()};
}

// row of the padded pattern for row r = 2^len + m of the push kernels'
// per-length threshold table (full = 2^K - 1; rows 0, 1 and rows with
// len > K are unused)
__device__ __forceinline__ uint32_t padded_row(uint32_t r, uint32_t full) {
    const uint32_t len = 31u - (uint32_t)__clz((int)r);
    const uint32_t m = r - (1u << len);
    return (m | ((m & 1u) ? ~((1u << len) - 1u) : 0u)) & full;
}

template <int kTab, bool kClust = false>
__device__ __forceinline__ void load_push_tables(const PushLds &L, const uint32_t *thr, const int64_t *gfx,
                                                 const int64_t *gpad, int tau, int tid, int NT, uint32_t full) {
    if (kClust) {
        for (int i = tid; i < kClustThrRows * kMaxL; i += NT) L.thr[i] = thr[tau * kClustThrRows * kMaxL + i];
        for (int i = tid; i < kClustGfxRows * kMaxL; i += NT) L.gfx[i] = gfx[tau * kClustGfxRows * kMaxL + i];
        for (int i = tid; i < kClustGpad; i += NT) L.gpad[i] = gpad[tau * kClustGpad + i];
        return;
    }
    for (int i = 2 * kMaxL + tid; i < kThrRows * kMaxL; i += NT)
        L.thr[i] = thr[(tau * kPatterns + (int)padded_row((uint32_t)(i / kMaxL), full)) * kMaxL + i % kMaxL];
    const int64_t *rows = gfx + (size_t)tau * kHidMasks * kRowWords;
    if (kTab == kBucketPush) {
        for (int i = tid; i < kHidMasks * kRowWords; i += NT) L.gfx[i] = rows[i];
    } else if (kTab == kBucketMid) {
        for (int i = tid; i < kHidMasks * kMaxL; i += NT) L.gfx[i] = rows[(i / kMaxL) * kRowWords + i % kMaxL];
    }
}

// Gather of a clause's literal values: bit k of the result is the value of
// the variable of slot k (polarity not applied), for slots 0..len-1.
template <int LEN>
__device__ __forceinline__ uint32_t gather_fixed(const uint8_t *v, const uint4 &r) {
    const uint32_t e[7] = {r.x, r.x >> 16, r.y, r.y >> 16, r.z, r.z >> 16, r.w};
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < LEN; ++k) m |= (uint32_t)v[e[k] & 0x7fffu] << k;
    return m;
}

// Padding positions of a clause of len literals, filled with copies of
// literal 0: up to the table width (full = 2^K - 1) in the padded model, up to
// K = max(len, 3) in the size-clustered one.
template <bool kClust>
__device__ __forceinline__ uint32_t pad_mask(uint32_t len, uint32_t full) {
    const uint32_t top = kClust ? (1u << (len < 3u ? 3u : len)) - 1u : full;
    return top & ~((1u << len) - 1u);
}

// negation bits of a record of LEN literals (the record's last word)
template <int LEN>
__device__ __forceinline__ uint32_t neg_bits(const uint4 &r) {
    return LEN < 7 ? r.w & ((1u << LEN) - 1u) : r.w >> 19;
}

// literal-truth pattern of a clause of LEN literals, padding filled
template <int LEN, bool kClust>
__device__ __forceinline__ uint32_t pattern_fixed(const uint8_t *v, const uint4 &r, uint32_t full) {
    const uint32_t m = gather_fixed<LEN>(v, r) ^ neg_bits<LEN>(r);
    return m | (pad_mask<kClust>((uint32_t)LEN, full) & (0u - (m & 1u)));
}

// Scatter of a clause's contributions: g0 (the merged slot 0) to slot 0's
// variable, gr[k] to slot k's for k = 1..len-1.
template <int k, int LEN>
__device__ __forceinline__ void scatter_slots(int64_t *x, const uint4 &r, const int64_t (&g)[8]) {
    if constexpr (k < LEN) {
        push_add(x, slot_var<k>(r), slot_neg<k>(r), g[k]);
        scatter_slots<k + 1, LEN>(x, r, g);
    }
}

__device__ __forceinline__ int64_t buffer_load_i64(__amdgpu_buffer_rsrc_t rs, int off) {
    return __builtin_bit_cast(int64_t, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
}

// The contributions of hidden mask n to a clause of LEN literals: g[0] the
// merged one of slot 0 (with its padding copies), g[k] slot k's.  All of them
// are read before the first accumulator update: the compiler cannot tell
// that the atomics never touch the tables, so reads placed after an atomic
// would each wait for it.
template <int LEN, int kTab>
__device__ __forceinline__ void table_reads(const PushLds &L, uint32_t n, int64_t (&g)[8]) {
    const int off = (int)n * (kRowWords * 8);
    if (kTab == kBucketPush) {
        const int64_t *row = L.gfx + n * kRowWords;
        g[0] = row[kMaxL + LEN];
#pragma unroll
        for (int k = 1; k < LEN; ++k) g[k] = row[k];
    } else if (kTab == kBucketMid) {
        const int64_t *row = L.gfx + n * kMaxL;
        g[0] = buffer_load_i64(L.grs, off + (kMaxL + LEN) * 8);
#pragma unroll
        for (int k = 1; k < LEN; ++k) g[k] = row[k];
    } else {
        g[0] = buffer_load_i64(L.grs, off + (kMaxL + LEN) * 8);
#pragma unroll
        for (int k = 1; k < LEN; ++k) g[k] = buffer_load_i64(L.grs, off + k * 8);
    }
}

// cnt += (m != Z) as one compare and one add-with-carry, issued where m is
// made; in the plain C form the compiler recomputes m from its parts at the
// end of the clause (three instructions).  Z <= 64 (an inline constant).
template <uint32_t Z>
__device__ __forceinline__ void count_satisfied(int &cnt, uint32_t m) {
    static_assert(Z <= 64u, "the compare takes an inline constant");
    asm volatile("v_cmp_ne_u32 vcc, %2, %1\n\tv_addc_co_u32 %0, vcc, 0, %0, vcc" : "+v"(cnt) : "v"(m), "i"(Z) : "vcc");
}

// One clause of compile-time length LEN: gather, literal-truth pattern,
// count; when sampling, the hidden draw and the scatter of its
// contributions into the LDS accumulators.  Adds 1 to cnt if it is
// satisfied.
// kClust: the size-clustered model; a clause of length len takes the tables
// of group K = max(len, 3) (L = 3 or K + 1 hidden units, drawn from blocks
// 2c and, for L > 4, 2c + 1), and nbh, full and lmask are unused.
template <int LEN, bool kSample, bool kClust, int NB, int kTab>
__device__ __forceinline__ void clause_one(const PushLds &L, const uint4 &r, uint32_t oc, const PhiloxSweep &ps,
                                           Key2 key, uint32_t nbh, uint32_t full, uint32_t lmask, int &cnt) {
    // size-clustered model: the padded pattern.  Padded model: the pattern of
    // the LEN literals alone, whose threshold row 2^LEN + m holds the padded
    // pattern's; for LEN < 7 the record's last word is the negation bits |
    // 2^LEN, so one XOR makes the row itself (a clause is satisfied iff its
    // row is not 2^LEN).
    constexpr bool kRow = !kClust && LEN < 7;
    const uint32_t m = kClust  ? pattern_fixed<LEN, kClust>(L.v, r, full)
                       : kRow ? gather_fixed<LEN>(L.v, r) ^ r.w
                              : gather_fixed<LEN>(L.v, r) ^ neg_bits<LEN>(r);
    count_satisfied<kRow ? (1u << LEN) : 0u>(cnt, m);
    if (kSample) {
        int64_t g[8];
        if (kClust) {
            constexpr uint32_t Kc = LEN < 3 ? 3u : (uint32_t)LEN;
            constexpr bool big = Kc > 3u;                            // L = K + 1 > 4: two blocks
            const uint32_t n = hidden_mask<big ? 2 : 1>(L.thr + ((1u << Kc) - 8u + m) * kMaxL, oc, ps, key, 0u) &
                               (big ? (2u << Kc) - 1u : 7u);
            const int64_t *gr = L.gfx + ((big ? (2u << Kc) - 24u : 0u) + n) * kMaxL;
            g[0] = L.gpad[(LEN <= 3 ? 8u * (LEN - 1u) : (2u << LEN) - 8u) + n];
#pragma unroll
            for (int k = 1; k < LEN; ++k) g[k] = gr[k];
        } else {
            // units at and above L (drawn, not masked) index rows that
            // repeat row n mod 2^L
            const uint32_t n = hidden_mask<NB>(L.thr + (kRow ? m : (1u << LEN) + m) * kMaxL, oc, ps, key, 0u);
            table_reads<LEN, kTab>(L, n, g);
        }
        scatter_slots<0, LEN>(L.x, r, g);
    }
}

// A wave's view of a range of clause records: raw buffer descriptors over
// the records and their first hidden-draw blocks, so a load of 64
// consecutive records takes a wave-uniform byte offset in a scalar register
// and the lane's fixed offset in a vector register.  The lanes of a run's
// last step that lie past the run load the next records (or the zero
// records after the last formula's) and are masked.
struct RecView {
    __amdgpu_buffer_rsrc_t rec, orig;
};

__device__ __forceinline__ RecView rec_view(const uint4 *rec, const uint32_t *orig, int M) {
    return RecView{__builtin_amdgcn_make_buffer_rsrc(const_cast<uint4 *>(rec), (short)0, M * 16, kRawBufferWord3),
                   __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(orig), (short)0, M * 4, kRawBufferWord3)};
}

// Keeps every word of a loaded record, and its first Philox block, in
// registers of its own until the record's clause runs.  A word the clause
// length leaves unused would otherwise be given to a temporary of the clause
// before it, and writing that temporary waits for the prefetch to land.
__device__ __forceinline__ void rec_hold(const uint4 &r, uint32_t oc) {
    asm volatile("" ::"v"(r.x), "v"(r.y), "v"(r.z), "v"(r.w), "v"(oc));
}

__device__ __forceinline__ void rec_load(const RecView &rv, int first, int lane, uint4 &r, uint32_t &oc) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rv.rec, lane * 16, first * 16, 0);
    r = make_uint4(v[0], v[1], v[2], v[3]);
    oc = __builtin_amdgcn_raw_buffer_load_b32(rv.orig, lane * 4, first * 4, 0);
}

// Steps of 64 consecutive records, taken by the waves from a workgroup-wide
// counter in LDS.  The runs of the clause lengths are cut into steps and
// numbered in order (run of length 1 first); a wave takes the next step
// number whenever it starts one, so the waves that the SIMDs serve first
// simply take more steps and all of them reach the end of the clause phase
// together (fixed shares left the youngest waves running alone at the end of
// every clause phase).  The accumulators are exact integers, so which wave
// takes which step does not change any result.  The counter hands out pairs
// of consecutive steps (2j, 2j + 1): a wave goes to the counter only every
// other step, so half as often waits for the add's result, whose wait also
// covers the previous clause's accumulator atomics.  The counter runs on
// across the sweeps of an item.  Of T steps (ceil(T/2) pairs) and W waves,
// every wave takes one pair past the last one per sweep, except, for odd T,
// the wave holding the last pair, whose second number T already ends its
// clause phase: sweep s of an item owns the pair numbers [s P, (s + 1) P)
// with P = ceil(T/2) + W - (T mod 2).
// With dyn == 0 the steps are dealt round-robin instead (step k to wave
// k mod W, no counter): better when another workgroup shares the CU and
// fills the SIMDs while this one waits at its barrier.
struct StepCounter {
    int base;                    // first pair number of this sweep
    int dyn;                     // 1: take steps from the counter; 0: round-robin
    int wave, nw;
};

// LDS byte address of the step counter (word 62 of the layout's counts,
// zeroed before an item's first sweep); the sweep kernels have no static
// LDS, so their dynamic LDS starts at address 0
template <int kTab, bool kClust>
constexpr int step_counter_addr() {
    return (kClust ? kClustCntOff
                   : kTab == kBucketWide ? kWideCntOff : kTab == kBucketMid ? kMidCntOff : kPushCntOff) + 62 * 4;
}

// One LDS add-and-return of 1 for the wave, by lane 0 alone, its result
// returned to every lane in a scalar register.  The compiler's atomic form
// wraps an add at a uniform address in a whole-wave reduction (lane counts,
// prefix, two broadcasts: 8 VALU instructions per step, i.e. per clause), and
// a branch on lane 0 costs a zeroed result register, the address moved into a
// vector register and the exec-mask save and restore around it.  Here one
// asm block narrows exec to lane 0, issues the add, waits for its result
// (so the returned register is never read early), restores exec and reads
// lane 0.  The address is the register holding the added 1 plus the
// instruction's offset (kAddr - 1), so no register is set up per step.  The
// whole wave must be active (lane 0 in exec).
template <int kAddr>
__device__ __forceinline__ int lds_fetch_add1_wave(uint32_t one) {
    static_assert(kAddr >= 1 && kAddr <= 65536, "the offset field holds 16 bits");
    int k;
    uint64_t saved;
    uint32_t r;
    asm volatile(
        "s_mov_b64 %1, exec\n\t"
        "s_mov_b64 exec, 1\n\t"
        "ds_add_rtn_u32 %2, %3, %3 offset:%4\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_mov_b64 exec, %1\n\t"
        "v_readfirstlane_b32 %0, %2"
        : "=s"(k), "=&s"(saved), "=&v"(r)
        : "v"(one), "i"(kAddr - 1)
        : "memory");
    return k;
}

template <int kAddr>
__device__ __forceinline__ int take_step(const StepCounter &sc, int prev) {
    if (!sc.dyn) return prev < 0 ? sc.wave : prev + sc.nw;
    if (prev >= 0 && (prev & 1) == 0) return prev + 1;     // the second step of the pair
    return 2 * (lds_fetch_add1_wave<kAddr>(1u) - sc.base);
}

// The steps [olo, ohi) of the run [lo, hi) of clauses of length LEN.  `k`
// is the wave's current step number: if it is in this run, the wave
// processes it and keeps taking steps until it gets one past the run, which
// it leaves in `k` for the next run.  The next step's records are loaded
// while the current ones are processed (two register sets, no copies).  The
// load is issued on every iteration, past the run's end from the current
// step again (its values are never used), so the wait for a step's records
// counts the one load issued after them on every path.
template <int LEN, bool kSample, bool kClust, int NB, int kTab>
__device__ __forceinline__ int clause_segment(const PushLds &L, const RecView &rv, int lo, int hi, int olo, int ohi,
                                              int &k, const StepCounter &sc, int lane, const PhiloxSweep &ps,
                                              Key2 key, uint32_t nbh, uint32_t full, uint32_t lmask) {
    int cnt = 0;
    if (k >= ohi) return 0;
    int base = lo + (k - olo) * kWave;
    uint4 ra, rb;
    uint32_t oa, ob;
    rec_load(rv, base, lane, ra, oa);
    for (;;) {
        int kn = take_step<step_counter_addr<kTab, kClust>()>(sc, k);
        int next = lo + (kn - olo) * kWave;
        rec_load(rv, kn < ohi ? next : base, lane, rb, ob);
        rec_hold(ra, oa);
        if (lane < hi - base) clause_one<LEN, kSample, kClust, NB, kTab>(L, ra, oa, ps, key, nbh, full, lmask, cnt);
        k = kn;
        if (kn >= ohi) break;
        base = next;
        kn = take_step<step_counter_addr<kTab, kClust>()>(sc, k);
        next = lo + (kn - olo) * kWave;
        rec_load(rv, kn < ohi ? next : base, lane, ra, oa);
        rec_hold(rb, ob);
        if (lane < hi - base) clause_one<LEN, kSample, kClust, NB, kTab>(L, rb, ob, ps, key, nbh, full, lmask, cnt);
        k = kn;
        if (kn >= ohi) break;
        base = next;
    }
    return cnt;
}

// steps of the runs of a range: o[k] = steps of the runs of lengths < k + 1
__device__ __forceinline__ void run_steps(const int32_t (&bnd)[8], int32_t (&o)[8]) {
    o[0] = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k) o[k] = o[k - 1] + (bnd[k] - bnd[k - 1] + kWave - 1) / kWave;
}

// Clause phase over the M records of a range (a formula's, or a split
// member's run), sorted by clause length with bnd[k] = the number of records
// of length <= k (bnd[0] = 0, bnd[7] = M).  The waves walk the records
// length by length in steps of 64 (above), so every step is one clause
// length (the gather and scatter unrolled for it) with no per-record length
// test.  Returns this thread's number of satisfied clauses.
template <bool kSample, bool kClust, int NB, int kTab>
__device__ __forceinline__ int clause_phase_nb(const PushLds &L, const RecView &rv, const int32_t (&bnd)[8],
                                               const StepCounter &sc, int lane, const PhiloxSweep &ps, Key2 key,
                                               uint32_t nbh, uint32_t full, uint32_t lmask) {
    int32_t o[8];
    run_steps(bnd, o);
    int cnt = 0;
    int k = take_step<step_counter_addr<kTab, kClust>()>(sc, -1);
#define HP_SEG(LEN)                                                                                              \
    cnt += clause_segment<LEN, kSample, kClust, NB, kTab>(L, rv, bnd[LEN - 1], bnd[LEN], o[LEN - 1], o[LEN], k,  \
                                                          sc, lane, ps, key, nbh, full, lmask)
    HP_SEG(1);
    HP_SEG(2);
    HP_SEG(3);
    HP_SEG(4);
    HP_SEG(5);
    HP_SEG(6);
    HP_SEG(7);
#undef HP_SEG
    return cnt;
}

// counter numbers (pairs of steps) one sweep of a range consumes
__device__ __forceinline__ int sweep_step_numbers(const int32_t (&bnd)[8], int NT) {
    int32_t o[8];
    run_steps(bnd, o);
    return (o[7] + 1) / 2 + NT / kWave - (o[7] & 1);
}

template <bool kSample, bool kClust, int kTab>
__device__ __forceinline__ int clause_phase(const PushLds &L, const uint4 *__restrict__ rec,
                                            const uint32_t *__restrict__ orig, int M, const int32_t (&bnd)[8],
                                            const StepCounter &sc, int tid, const PhiloxSweep &ps, Key2 key,
                                            uint32_t nbh, uint32_t full, uint32_t lmask) {
    const int lane = tid & (kWave - 1);
    const RecView rv = rec_view(rec, orig, M);
    if (kClust) return clause_phase_nb<kSample, kClust, 0, kTab>(L, rv, bnd, sc, lane, ps, key, nbh, full, lmask);
    return nbh > 1 ? clause_phase_nb<kSample, kClust, 2, kTab>(L, rv, bnd, sc, lane, ps, key, nbh, full, lmask)
                   : clause_phase_nb<kSample, kClust, 1, kTab>(L, rv, bnd, sc, lane, ps, key, nbh, full, lmask);
}

// Range-relative length bounds of split member g of G: the member's run
// holds the sorted records g, g + G, g + 2G, ..., so of the lofs[k] records
// of length <= k it holds ceil((lofs[k] - g) / G).
__device__ __forceinline__ void member_bounds(const int32_t (&lofs)[8], int g, int G, int32_t (&bnd)[8]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) bnd[k] = lofs[k] > g ? (lofs[k] - g + G - 1) / G : 0;
}

// ---- mixed precision: the per-clause products on MFMA ---------------------
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

// 8 binary inputs (bit i of `bits`) as BF16 0.0 / 1.0, element i = input i
__device__ __forceinline__ bf16x8_t bits_bf16x8(uint32_t bits) {
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t lo = (uint32_t)((int32_t)(bits << (31 - 2 * j)) >> 31);       // 0 or ~0
        const uint32_t hi = (uint32_t)((int32_t)(bits << (30 - 2 * j)) >> 31);
        w[j] = (lo & 0x00003F80u) | (hi & 0x3F800000u);
    }
    return __builtin_bit_cast(bf16x8_t, make_uint4(w[0], w[1], w[2], w[3]));
}

__device__ __forceinline__ int64_t shfl_xor_i64(int64_t v, int m) {
    const int lo = __shfl_xor((int)(uint32_t)v, m, 64), hi = __shfl_xor((int)(v >> 32), m, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Hidden-draw margin: |p32 - p| <= 3e-7 for the FP32 logit (sum of four
// exact limb-pair products) and the FP32 sigmoid (v_exp_f32, v_rcp_f32);
// a draw whose U lies within 16 * 2^-24 (9.5e-7) of p32 is taken from the
// FP64 threshold table instead, so every hidden bit equals the FP64 rule.
constexpr float kDrawMargin24 = 16.0f;

// Clause phase with the two per-clause contractions on MFMA.  A wave takes
// 32 clauses at a time; lane l works on clause tb + l % 32, lanes l and l+32
// on the same clause: the low half draws hidden units 0..3 (Philox block
// 2c) and scatters slots 0..3, the high half units 4..7 (block 2c+1) and
// slots 4..6.  The MFMA result lands in that layout (register i = limb pair
// i / 4 of unit or slot 4h + i % 4), so the limb pairs are summed in
// registers.  Counts, hidden bits and fixed-point contributions equal the
// table path's.
template <bool kSample>
__device__ __forceinline__ int clause_phase_mfma(const PushLds &L, const uint4 *__restrict__ rec,
                                                 const uint32_t *__restrict__ orig, int C, int tid, int NT,
                                                 uint32_t tlo, uint32_t thi, uint32_t chain, Key2 key,
                                                 uint32_t nbh, uint32_t full, uint32_t lmask, int K,
                                                 bf16x8_t a1, bf16x8_t a2, double inv_scale) {
    const int lane = tid & (kWave - 1), wave = tid / kWave, n_waves = NT / kWave;
    const int half = lane >> 5;
    int cnt = 0;
    for (int tb = wave * 32; tb < C; tb += n_waves * 32) {      // uniform over the wave
        const int c = tb + (lane & 31);
        const bool act = c < C;
        uint4 r = make_uint4(0, 0, 0, 0);
        uint32_t oc = 0;
        if (act) {
            r = rec[c];
            oc = orig[c];
        }
        const uint32_t len = act ? rec_len(r.w) : 0u;
        const uint32_t negm = act ? rec_negm(r.w) : 0u;
        const uint32_t e[7] = {r.x & 0xffffu, r.x >> 16, r.y & 0xffffu, r.y >> 16,
                               r.z & 0xffffu, r.z >> 16, r.w & 0xffffu};
        uint32_t m = 0;
        if (act) {
            m = L.v[e[0] & 0x7fffu];
            if (len > 1) m |= (uint32_t)L.v[e[1] & 0x7fffu] << 1;
            if (len > 2) m |= (uint32_t)L.v[e[2] & 0x7fffu] << 2;
            if (len > 3) m |= (uint32_t)L.v[e[3] & 0x7fffu] << 3;
            if (len > 4) m |= (uint32_t)L.v[e[4] & 0x7fffu] << 4;
            if (len > 5) m |= (uint32_t)L.v[e[5] & 0x7fffu] << 5;
            if (len > 6) m |= (uint32_t)L.v[e[6] & 0x7fffu] << 6;
            m ^= negm;
            m |= (m & 1u) ? (full & ~((1u << len) - 1u)) : 0u;
            if (half == 0) cnt += (m != 0u);
        }
        if (!kSample) continue;
        // ---- hidden logits z = b + W^T lit, limb pairs summed in FP32 ----
        const f32x16_t d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bits_bf16x8(act ? (m | 0x80u) : 0u),
                                                                    f32x16_t{}, 0, 0, 0);
        const uint4 rw = philox4x32_10(make_uint4(tlo, chain, kPhaseHidden | (oc + (uint32_t)half), thi), key);
        const uint32_t w4[4] = {rw.x, rw.y, rw.z, rw.w};
        uint32_t nh = 0, amb = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float z = ((d1[q] + d1[4 + q]) + d1[8 + q]) + d1[12 + q];
            const float p = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
            const float d = fmaf(p, -16777216.0f, (float)(w4[q] >> 8));   // (U - p) 2^24
            nh |= (d < 0.0f ? 1u : 0u) << q;
            amb |= (fabsf(d) <= kDrawMargin24 ? 1u : 0u) << q;
        }
        if (amb != 0u && act) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if ((amb >> q) & 1u) {
                    const uint32_t row = (1u << len) + (m & ((1u << len) - 1u));
                    const uint32_t bit = w4[q] <= L.thr[row * kMaxL + 4 * half + q] ? 1u : 0u;
                    nh = (nh & ~(1u << q)) | (bit << q);
                }
        }
        const uint32_t other = (uint32_t)__shfl_xor((int)nh, 32, 64);
        const uint32_t n = act ? ((half ? (other | (nh << 4)) : (nh | (other << 4))) & lmask) : 0u;
        // ---- contributions l = W h, limb pairs summed in FP64, fixed point ----
        const f32x16_t d2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, bits_bf16x8(n), f32x16_t{}, 0, 0, 0);
        int64_t fx[4], pad = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * half + q;
            const double lk = (((double)d2[q] + (double)d2[4 + q]) + (double)d2[8 + q]) + (double)d2[12 + q];
            fx[q] = k < K ? (int64_t)llrint(lk * inv_scale) : 0;
            if (k >= (int)len && k < K) pad += fx[q];    // padding copies of literal 0
        }
        pad += shfl_xor_i64(pad, 32);
        if (act) {
            if (half == 0) {
                push_add(L.x, e[0], fx[0] + pad);
#pragma unroll
                for (int q = 1; q < 4; ++q)
                    if (q < (int)len) push_add(L.x, e[q], fx[q]);
            } else {
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if (4 + q < (int)len) push_add(L.x, e[4 + q], fx[q]);
            }
        }
    }
    return cnt;
}

template <typename Real>
__device__ __forceinline__ Real buffer_load_real(__amdgpu_buffer_rsrc_t rs, int i);
template <>
__device__ __forceinline__ float buffer_load_real<float>(__amdgpu_buffer_rsrc_t rs, int i) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, i * 4, 0, 0));
}
typedef __attribute__((__vector_size__(2 * sizeof(uint32_t)))) uint32_t u32x2_t;
template <>
__device__ __forceinline__ double buffer_load_real<double>(__amdgpu_buffer_rsrc_t rs, int i) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, i * 8, 0, 0));
}
__device__ __forceinline__ void buffer_store_real(float v, __amdgpu_buffer_rsrc_t rs, int i) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, i * 4, 0, 0);
}
__device__ __forceinline__ void buffer_store_real(double v, __amdgpu_buffer_rsrc_t rs, int i) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), rs, i * 8, 0, 0);
}

// Visible update of one variable from its fixed-point logit: sigmoid, EMA,
// Bernoulli draw U < rho with U = (word >> 8) 2^-24.
template <typename Real>
__device__ __forceinline__ uint8_t visible_update(int64_t xi, double fx_scale, Real &nu, Real alpha,
                                                  uint32_t word) {
    const Real x = (Real)((double)xi * fx_scale);
    const Real rho = sigmoid(x);
    nu = ema(nu, rho, alpha);
    return (Real(word >> 8) * Real(1.0 / 16777216.0)) < rho ? 1 : 0;
}

// The FP32 form: -x log2(e) from the two 32-bit halves of the fixed-point
// sum (single-rate conversions with the scale and -log2(e) folded into the
// two constants; about 2^-23 |x| error), the logistic function from the
// hardware exp2 and reciprocal (about 2 ulp more relative in exp(-x), so
// |d rho| <= 0.25 of that: below 4e-7 for |x| <= 20), the moving average
// and the draw in FP32.  The reciprocal is taken of (1 + e^-x) 2^-24, which
// gives 2^24 rho with the same rounding as rho itself (a power-of-two
// scale), so the draw compares the 24-bit uniform integer with it directly
// and the average uses alpha 2^-48 (2^24 rho)(2^24 - 2^24 rho).
template <>
__device__ __forceinline__ uint8_t visible_update<float>(int64_t xi, double fx_scale, float &nu, float alpha,
                                                         uint32_t word) {
    const float sc = (float)(fx_scale * -1.4426950408889634);  // -log2(e) 2^-S
    const float y = fmaf((float)(int32_t)(xi >> 32), sc * 4294967296.0f, (float)(uint32_t)xi * sc);
    const float rho24 = __builtin_amdgcn_rcpf(fmaf(__builtin_amdgcn_exp2f(y), 0x1p-24f, 0x1p-24f));
    nu = fmaf(alpha * 0x1p-48f * rho24, 16777216.0f - rho24, (1.0f - alpha) * nu);
    return (float)(word >> 8) < rho24 ? 1 : 0;
}

// workgroup total of a per-thread count (uses L.cnt; ends with a barrier)
__device__ __forceinline__ int block_total(const PushLds &L, int cnt, int tid, int NT) {
    cnt = wave_sum(cnt);
    if ((tid & (kWave - 1)) == 0) L.cnt[tid / kWave] = cnt;
    __syncthreads();
    int total = 0;
    for (int wv = 0; wv < NT / kWave; ++wv) total += L.cnt[wv];
    return total;
}

// One chain per workgroup at a time.  Q.ctr == nullptr: workgroup w runs
// item w.  Otherwise the grid is persistent: workgroups take items from
// atomic counters (zeroed before the launch), largest formulas first, so
// uneven sizes balance over the resident grid.  The items are grouped by
// XCD (whole formulas, balanced by work): a workgroup drains its own XCD's
// range first, so the workgroups that share an L2 run the chains of the same
// few formulas and their clause records stay in that L2, then it helps the
// other ranges in turn.
template <typename Real, int VPT, int kTab, bool kMfma = false, bool kClust = false>
__global__ __launch_bounds__(1024) void sweep_push_kernel(SweepParams<Real> P, WorkQueue Q) {
    extern __shared__ __align__(16) unsigned char lds[];
    int *s_item = reinterpret_cast<int *>(lds + (kClust                  ? kClustCntOff
                                                 : kTab == kBucketWide ? kWideCntOff
                                                 : kTab == kBucketMid  ? kMidCntOff
                                                                       : kPushCntOff)) +
                  63;
    const int tid = threadIdx.x, NT = blockDim.x;
    const bool sample = P.n_sweeps > 0;
    const int64_t S = sample ? P.n_sweeps : 1;
    const uint32_t nbh = (uint32_t)(P.L + 3) >> 2;
    const uint32_t full = (1u << P.K) - 1u;
    const uint32_t lmask = (1u << P.L) - 1u;
    const Real alpha = P.alpha;
    const double fx_scale = P.fx_scale;
    const int64_t t0 = *P.t_ptr;

    const int home = (int)(blockIdx.x % kXcds);
    const int wave_id = __builtin_amdgcn_readfirstlane(tid / kWave);
    int qx = 0;                       // thread 0: ranges drained so far (own XCD first)
    for (int it = 0;; ++it) {
        int item;
        if (Q.ctr == nullptr) {
            if (it > 0) break;
            item = blockIdx.x;
        } else {
            if (tid == 0) {
                int got = -1;
                for (; qx < kXcds; ++qx) {
                    const int x = (home + qx) % kXcds;
                    const int n = Q.xq[x + 1] - Q.xq[x];
                    if (n <= 0) continue;
                    const uint32_t k = atomicAdd(Q.ctr + 32 * x, 1u);
                    if (k < (uint32_t)n) {
                        got = Q.xq[x] + (int)k;
                        break;
                    }
                }
                *s_item = got;
            }
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(*s_item);    // the same for every thread
            __syncthreads();          // s_item is rewritten by the next take
            if (item < 0) break;
        }
        const WorkItem w = P.work[item];
        const FormulaDev fd = P.fd[w.f];
        const int N = fd.n, C = fd.c;
        const int tau = P.temp_of_chain[(int64_t)w.f * P.B + w.b];
        const PushLds L = kClust ? push_lds_clust(lds, P.lds_x_off)
                                 : push_lds_for<kTab>(lds, P.lds_x_off, P.gfx, tau);
        const int64_t sbase = fd.var_off * P.B + (int64_t)w.b * N;
        const uint4 *__restrict__ rec = P.rec + fd.clause_off;
        const uint32_t *__restrict__ orig = P.orig + fd.clause_off;
        const Key2 key{P.key0, P.key1 ^ (uint32_t)w.f};
        const int32_t *__restrict__ negcnt = P.negcnt + fd.var_off;

        load_push_tables<kTab, kClust>(L, P.thr, P.gfx, P.gpad, tau, tid, NT, full);
        for (int i = tid; i < N; i += NT) {
            L.v[i] = P.v[sbase + i];
            L.x[i] = negcnt[i];
        }
        bf16x8_t a1 = {}, a2 = {};
        if (kMfma) {
            a1 = __builtin_bit_cast(bf16x8_t, P.mfma[((size_t)tau * 2 + 0) * kWave + (tid & (kWave - 1))]);
            a2 = __builtin_bit_cast(bf16x8_t, P.mfma[((size_t)tau * 2 + 1) * kWave + (tid & (kWave - 1))]);
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
        // buffer views of this chain's best and nu and the formula's negated-
        // slot counts: the visible phase addresses them by the variable's
        // offset alone (accesses past N read zeros and write nothing)
        const __amdgpu_buffer_rsrc_t best_rs =
            __builtin_amdgcn_make_buffer_rsrc(P.best + sbase, (short)0, N, kRawBufferWord3);
        const __amdgpu_buffer_rsrc_t nu_rs =
            __builtin_amdgcn_make_buffer_rsrc(P.nu + sbase, (short)0, N * (int)sizeof(Real), kRawBufferWord3);
        const __amdgpu_buffer_rsrc_t neg_rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t *>(negcnt), (short)0, N * 4, kRawBufferWord3);
        int smax = P.s_max[(int64_t)w.f * P.B + w.b];
        const int steps = sweep_step_numbers(fd.lofs, NT);     // step numbers per sweep
        if (tid == 0) L.cnt[62] = 0;
        __syncthreads();

        for (int64_t s = 0; s < S; ++s) {
            const uint64_t t = (uint64_t)(t0 + s);
            const uint32_t tlo = (uint32_t)t, thi = (uint32_t)(t >> 32);
            const PhiloxSweep ps = philox_sweep_consts(tlo, (uint32_t)w.b, thi, key);
            int cnt;
            if (kMfma)
                cnt = sample ? clause_phase_mfma<true>(L, rec, orig, C, tid, NT, tlo, thi, (uint32_t)w.b, key, nbh, full,
                                                       lmask, P.K, a1, a2, 1.0 / fx_scale)
                             : clause_phase_mfma<false>(L, rec, orig, C, tid, NT, tlo, thi, (uint32_t)w.b, key, nbh,
                                                        full, lmask, P.K, a1, a2, 1.0 / fx_scale);
            else
            {
                const StepCounter sc{(int)s * steps, P.dyn_steps, wave_id, NT / kWave};
                cnt = sample ? clause_phase<true, kClust, kTab>(L, rec, orig, C, fd.lofs, sc, tid, ps, key, nbh, full, lmask)
                             : clause_phase<false, kClust, kTab>(L, rec, orig, C, fd.lofs, sc, tid, ps, key, nbh, full, lmask);
            }
            const int total = block_total(L, cnt, tid, NT);
            const bool improved = total > smax;
            if (improved) smax = total;
            // ---- visible phase ----
            const int groups = (N + 3) >> 2;
            const int jmax = VPT > 0 ? VPT : (groups + NT - 1) / NT;
            // the thread index passes through an empty asm each sweep, so the
            // per-variable offsets below are recomputed here instead of being
            // hoisted out of the sweep loop into registers held across the
            // clause phase
            int vtid = tid;
            asm volatile("" : "+v"(vtid));
#pragma unroll
            for (int j = 0; j < (VPT > 0 ? VPT : 1); ++j) {
              for (int jj = (VPT > 0 ? j : 0); jj < (VPT > 0 ? j + 1 : jmax); ++jj) {
                const int grp = vtid + jj * NT;
                if (grp < groups) {
                    uint4 r = make_uint4(0, 0, 0, 0);
                    int32_t nc[4] = {0, 0, 0, 0};
                    if (sample) {
                        r = philox_sweep(kPhaseVisible | (uint32_t)grp, ps, key);
                        // the accumulators restart at the negated-slot counts
                        const auto c4 = __builtin_amdgcn_raw_buffer_load_b128(neg_rs, grp * 16, 0, 0);
                        nc[0] = (int32_t)c4[0], nc[1] = (int32_t)c4[1], nc[2] = (int32_t)c4[2], nc[3] = (int32_t)c4[3];
                    }
                    const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int i = grp * 4 + q;
                        if (i < N) {
                            if (improved) __builtin_amdgcn_raw_buffer_store_b8(L.v[i], best_rs, i, 0, 0);
                            if (sample) {
                                const int64_t xi = L.x[i];
                                L.x[i] = nc[q];
                                if (VPT > 0) {
                                    L.v[i] = visible_update(xi, fx_scale, nu[j][q], alpha, rw[q]);
                                } else {
                                    Real nv = buffer_load_real<Real>(nu_rs, i);
                                    L.v[i] = visible_update(xi, fx_scale, nv, alpha, rw[q]);
                                    buffer_store_real(nv, nu_rs, i);
                                }
                            }
                        }
                    }
                }
              }
            }
            __syncthreads();
        }
        for (int i = tid; i < N; i += NT) P.v[sbase + i] = L.v[i];
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
        __syncthreads();              // LDS is reused by the next item
    }
}

// --------------------------------------------------------------------------
// Split kernel: G co-resident workgroups per chain
// --------------------------------------------------------------------------
// Exchange between the G workgroups of one chain.  Partial logits, partial
// counts and new values cross workgroups through global memory with relaxed
// agent-scope atomic stores and loads: the stores write through and the loads
// miss the CU's vector cache and the per-XCD L2, so no cache-wide write-back
// or invalidation is needed (an agent-scope fence pair costs several
// microseconds on MI355X).  Workgroup-scope accesses served by a
// shared L2 are not an option for members on different CUs: outside
// thread-group-split mode the CU's vector cache may return a stale line, and
// the only invalidation that reaches it (buffer_inv sc1) also drops the L2's
// clean lines, which measured 3.7x slower per sweep.
__device__ __forceinline__ void xstore(int64_t *p, int64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t xload(const int64_t *p) {
    return __hip_atomic_load(const_cast<int64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void xstore(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t xload(const uint32_t *p) {
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void xstore(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t xload(const int32_t *p) {
    return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// State of one member of a split chain.
template <typename Real>
struct SplitCtx {
    PushLds L;
    const uint4 *rec;
    const uint32_t *orig;
    const int32_t *negcnt;
    int64_t *xpart;
    uint32_t *vbuf;
    int32_t *pcnt;
    int64_t sbase, nstride, S, t0;
    Key2 key;
    double fx_scale;
    Real alpha;
    int G, g, N, C, tid, NT, b, groups, q_lo, q_hi;
    int c_lo, c_hi;              // this member's run of records
    int32_t bnd[8];              // its records of length <= k, k = 0..7 (run-relative)
    int steps;                   // clause-phase step numbers per sweep
    uint32_t nbh, full, lmask;
    bool sample;
};

// Mailboxes of the exchange.  Every exchanged value carries a 2-bit tag, the
// sweep's tag 1 + (s mod 2) for local sweep s, and a reader waits until the
// word it loaded carries the tag of the sweep it is in; the buffers are
// zeroed (tag 0) before every launch.  A partial-logit or new-value slot
// holds the value of sweep s - 1 or s when a reader of sweep s looks at it,
// never s + 1: a member publishes the values of sweep s + 1 only after it has
// read every owner's new values of sweep s, which each owner publishes after
// it has read the partials (every member owns at least one variable group).
// The partial counts may be read after the new values are published, so they
// alternate between two slots by sweep parity and carry the tag
// 1 + (s div 2 mod 2): a slot is rewritten two sweeps later, only after every
// reader has passed the sweep in between.  The words themselves replace a
// counter barrier.
//   partial logit x (|x| < 2^61, bits 61..63 equal): x ^ (tag << 61)
//   partial count c (< 2^29): c | tag << 29
//   new values of a group: v0 | v1 << 8 | v2 << 16 | v3 << 24 | tag << 1
constexpr uint32_t kMailSpins = 1u << 20;   // default limit: ~1 s of waiting before giving up
constexpr int32_t kCntMask = (1 << 29) - 1;

__device__ __forceinline__ uint32_t tag_x(int64_t e) {
    const uint64_t u = (uint64_t)e;
    return (uint32_t)((u >> 61) & 3u) ^ (uint32_t)((u >> 63) * 3u);
}
__device__ __forceinline__ uint32_t tag_c(int32_t e) { return ((uint32_t)e >> 29) & 3u; }
__device__ __forceinline__ uint32_t tag_v(uint32_t w) { return (w >> 1) & 3u; }

// Reload *p until its tag is `want` (bounded: on time-out the error flag is
// raised and the stale word returned; once the flag is up nobody waits).
template <typename T, typename TagOf>
__device__ __forceinline__ T await_tag(const T *p, T e, uint32_t want, TagOf tag_of, int32_t *err,
                                       uint32_t limit) {
    uint32_t spins = 0;
    while (tag_of(e) != want) {
        __builtin_amdgcn_s_sleep(1);
        e = xload(p);
        if (++spins > limit) {
            xstore(err, 1);
            break;
        }
        if ((spins & 1023u) == 0u && xload(err)) break;
    }
    return e;
}

// The sweeps of one member.  Member g owns variable groups [q_lo, q_hi) (of
// 4): it keeps its own partial logits of those in LDS, publishes the others,
// sums the G partials of its own variables exactly (integers), draws their new
// values and publishes them; then every member reads the new values of the
// groups it does not own.  The owner's visible phase runs one variable per
// thread (variable own_lo + tid + j NT, j < VPT): the four threads of a group
// evaluate the group's Philox block alike and each takes its own word, and
// the group's first thread packs the four new values into the published word.
template <typename Real, int VPT, bool kClust>
__device__ __forceinline__ void split_sweeps(const SweepParams<Real> &P, const SplitParams &Q, const SplitCtx<Real> &c,
                                             Real (&nu)[VPT > 0 ? VPT : 1], const int32_t (&ncr)[VPT > 0 ? VPT : 1],
                                             int &smax) {
    const PushLds &L = c.L;
    const int G = c.G, g = c.g, N = c.N, tid = c.tid, NT = c.NT;
    const int own_lo = c.q_lo * 4, own_hi = min(N, c.q_hi * 4);
    const int jmax = VPT > 0 ? VPT : (own_hi - own_lo + NT - 1) / NT;
    for (int64_t s = 0; s < c.S; ++s) {
        const uint64_t t = (uint64_t)(c.t0 + s);
        const uint32_t tlo = (uint32_t)t, thi = (uint32_t)(t >> 32);
        const uint32_t tag = 1u + (uint32_t)(s & 1);
        // member g's records: every G-th of the length-sorted order (the same
        // mix of clause lengths for all members), stored as one contiguous run
        const PhiloxSweep ps = philox_sweep_consts(tlo, (uint32_t)c.b, thi, c.key);
        const StepCounter sc{(int)s * c.steps, 1, __builtin_amdgcn_readfirstlane(tid / kWave),
                             NT / kWave};
        const int cnt = c.sample ? clause_phase<true, kClust, kBucketPush>(L, c.rec + c.c_lo, c.orig + c.c_lo, c.c_hi - c.c_lo,
                                                              c.bnd, sc, tid, ps, c.key, c.nbh, c.full, c.lmask)
                                 : clause_phase<false, kClust, kBucketPush>(L, c.rec + c.c_lo, c.orig + c.c_lo, c.c_hi - c.c_lo,
                                                               c.bnd, sc, tid, ps, c.key, c.nbh, c.full, c.lmask);
        const int part = block_total(L, cnt, tid, NT);
        // publish the partial logits of the variables other members own
        if (c.sample) {
            for (int i = tid; i < N; i += NT) {
                if (i >= own_lo && i < own_hi) continue;
                xstore(&c.xpart[(size_t)g * c.nstride + i], L.x[i] ^ ((int64_t)tag << 61));
                L.x[i] = 0;
            }
        }
        int32_t *const pc = c.pcnt + (s & 1) * kMaxSplit;
        const uint32_t ctag = 1u + (uint32_t)((s >> 1) & 1);
        if (tid == 0) xstore(&pc[g], (int32_t)((uint32_t)part | (ctag << 29)));
        // the total count decides whether the counted state becomes the best;
        // with the owned variables' old values kept in registers (VPT > 0)
        // that wait moves behind the visible phase, off the critical path
        constexpr bool kLateCount = VPT > 0;
        // lane k < G of every wave fetches member k's count and the wave sums
        // them (one load per member and wave, not per thread)
        auto await_total = [&]() {
            const int lane = tid & (kWave - 1);
            int mine = 0;
            if (lane < G)
                mine = lane == g ? part : (await_tag(&pc[lane], xload(&pc[lane]), ctag, tag_c, Q.err, Q.wait_limit) & kCntMask);
            return wave_sum(mine);
        };
        bool improved = false;
        if (!kLateCount || !c.sample) {
            const int total = await_total();
            improved = total > smax;
            if (improved) smax = total;
        }
        uint8_t oldv[VPT > 0 ? VPT : 1];
        // visible phase on the owned variables
#pragma unroll
        for (int j = 0; j < (VPT > 0 ? VPT : 1); ++j) {
            for (int jj = (VPT > 0 ? j : 0); jj < (VPT > 0 ? j + 1 : jmax); ++jj) {
                const int i = own_lo + tid + jj * NT;
                const bool act = i < own_hi;
                uint32_t nvb = 0;
                if (VPT > 0) oldv[j] = act ? L.v[i] : 0;
                if (act) {
                    if (improved) P.best[c.sbase + i] = L.v[i];
                    if (c.sample) {
                        const uint4 r = philox_sweep(kPhaseVisible | (uint32_t)(i >> 2), ps, c.key);
                        const int q = i & 3;
                        const uint32_t word = q == 0 ? r.x : q == 1 ? r.y : q == 2 ? r.z : r.w;
                        // the partials of the other members: a batch of loads
                        // in flight before any is waited for
                        int64_t xs = (int64_t)(VPT > 0 ? ncr[j] : c.negcnt[i]) + L.x[i];
                        L.x[i] = 0;
                        for (int k0 = 0; k0 < G; k0 += 4) {
                            int64_t pk[4];
#pragma unroll
                            for (int kk = 0; kk < 4; ++kk) {
                                const int k = k0 + kk;
                                pk[kk] = (k < G && k != g) ? xload(&c.xpart[(size_t)k * c.nstride + i])
                                                           : ((int64_t)tag << 61);
                            }
#pragma unroll
                            for (int kk = 0; kk < 4; ++kk) {
                                const int k = k0 + kk;
                                if (k < G && k != g)
                                    pk[kk] = await_tag(&c.xpart[(size_t)k * c.nstride + i], pk[kk], tag, tag_x, Q.err, Q.wait_limit);
                                xs += pk[kk] ^ ((int64_t)tag << 61);
                            }
                        }
                        if (VPT > 0) {
                            nvb = visible_update(xs, c.fx_scale, nu[j], c.alpha, word);
                        } else {
                            Real nv = P.nu[c.sbase + i];
                            nvb = visible_update(xs, c.fx_scale, nv, c.alpha, word);
                            P.nu[c.sbase + i] = nv;
                        }
                        L.v[i] = (uint8_t)nvb;
                    }
                }
                if (c.sample) {
                    // own_lo and NT are multiples of 4: thread tid holds word i & 3 = tid & 3
                    const uint32_t b1 = __shfl_down(nvb, 1, kWave), b2 = __shfl_down(nvb, 2, kWave),
                                   b3 = __shfl_down(nvb, 3, kWave);
                    if (act && (tid & 3) == 0)
                        xstore(&c.vbuf[i >> 2], nvb | (b1 << 8) | (b2 << 16) | (b3 << 24) | (tag << 1));
                }
            }
        }
        if (kLateCount && c.sample) {
            const int total = await_total();
            if (total > smax) {
                smax = total;
#pragma unroll
                for (int j = 0; j < (VPT > 0 ? VPT : 1); ++j) {
                    const int i = own_lo + tid + j * NT;
                    if (i < own_hi) P.best[c.sbase + i] = oldv[j];
                }
            }
        }
        if (c.sample) {
            for (int q = tid; q < c.groups; q += NT) {
                if (q >= c.q_lo && q < c.q_hi) continue;
                const uint32_t word = await_tag(&c.vbuf[q], xload(&c.vbuf[q]), tag, tag_v, Q.err, Q.wait_limit);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (q * 4 + k < N) L.v[q * 4 + k] = (uint8_t)((word >> (8 * k)) & 1u);
            }
            __syncthreads();
        }
    }
}

template <typename Real, int VPT, bool kClust = false>
__global__ __launch_bounds__(1024) void sweep_split_kernel(SweepParams<Real> P, SplitParams Q) {
    extern __shared__ __align__(16) unsigned char lds[];
    SplitCtx<Real> c;
    c.L = kClust ? push_lds_clust(lds, P.lds_x_off) : push_lds(lds, P.lds_x_off);
    const PushLds &L = c.L;

    // workgroup -> (item, member g); with the XCD map the G members of an
    // item get workgroup ids congruent modulo the XCD count (same XCD under
    // round-robin dispatch, so they share the L2 that holds the formula)
    const int G = Q.G;
    int item, g;
    if (Q.xcd_map) {
        const int xcd = blockIdx.x % Q.n_xcd, slot = blockIdx.x / Q.n_xcd;
        item = (slot / G) * Q.n_xcd + xcd;
        g = slot % G;
    } else {
        item = blockIdx.x / G;
        g = blockIdx.x % G;
    }
    item = __builtin_amdgcn_readfirstlane(item);
    g = __builtin_amdgcn_readfirstlane(g);
    const WorkItem w = P.work[item];
    const FormulaDev fd = P.fd[w.f];
    const int N = fd.n;
    const int tid = threadIdx.x, NT = blockDim.x;
    const int tau = P.temp_of_chain[(int64_t)w.f * P.B + w.b];
    c.G = G;
    c.g = g;
    c.N = N;
    c.C = fd.c;
    c.c_lo = g * (fd.c / G) + min(g, fd.c % G);
    c.c_hi = c.c_lo + fd.c / G + (g < fd.c % G ? 1 : 0);
    member_bounds(fd.lofs, g, G, c.bnd);
    c.steps = sweep_step_numbers(c.bnd, NT);
    c.tid = tid;
    c.NT = NT;
    c.b = w.b;
    c.sbase = fd.var_off * P.B + (int64_t)w.b * N;
    c.rec = P.rec + fd.clause_off;
    c.orig = P.orig + fd.clause_off;
    c.key = Key2{P.key0, P.key1 ^ (uint32_t)w.f};
    c.sample = P.n_sweeps > 0;
    c.S = c.sample ? P.n_sweeps : 1;
    c.nbh = (uint32_t)(P.L + 3) >> 2;
    c.full = (1u << P.K) - 1u;
    c.lmask = (1u << P.L) - 1u;
    c.alpha = P.alpha;
    c.fx_scale = P.fx_scale;
    c.negcnt = P.negcnt + fd.var_off;
    c.nstride = Q.nstride;
    // this member's owned variable groups (of 4): a balanced partition, at
    // least one group each (the plan admits a split only if groups >= G)
    c.groups = (N + 3) >> 2;
    c.q_lo = (int)((int64_t)g * c.groups / G);
    c.q_hi = (int)((int64_t)(g + 1) * c.groups / G);
    // exchange buffers of this item (each starts on its own 128-byte line)
    c.xpart = Q.xpart + (size_t)item * G * Q.nstride;
    c.vbuf = reinterpret_cast<uint32_t *>(Q.vbuf + (size_t)item * Q.nstride);
    c.pcnt = Q.cnt + (size_t)item * 2 * kMaxSplit;

    load_push_tables<kBucketPush, kClust>(L, P.thr, P.gfx, P.gpad, tau, tid, NT, (1u << P.K) - 1u);
    for (int i = tid; i < N; i += NT) {
        L.v[i] = P.v[c.sbase + i];
        L.x[i] = 0;
    }
    // EMA and negation count of the owned variables own_lo + tid + j NT
    constexpr int VR = VPT > 0 ? VPT : 1;
    const int own_lo = c.q_lo * 4, own_hi = min(N, c.q_hi * 4);
    Real nu[VR];
    int32_t ncr[VR];
#pragma unroll
    for (int j = 0; j < VR; ++j) {
        const int i = own_lo + tid + j * NT;
        nu[j] = (VPT > 0 && i < own_hi) ? P.nu[c.sbase + i] : Real(0);
        ncr[j] = (VPT > 0 && i < own_hi) ? c.negcnt[i] : 0;
    }
    int smax = P.s_max[(int64_t)w.f * P.B + w.b];
    c.t0 = *P.t_ptr;
    if (tid == 0) L.cnt[62] = 0;           // the clause-phase step counter
    __syncthreads();

    split_sweeps<Real, VPT, kClust>(P, Q, c, nu, ncr, smax);

    // write back the owned part of the state
    for (int i = own_lo + tid; i < own_hi; i += NT) P.v[c.sbase + i] = L.v[i];
    if (VPT > 0) {
#pragma unroll
        for (int j = 0; j < VR; ++j) {
            const int i = own_lo + tid + j * NT;
            if (i < own_hi) P.nu[c.sbase + i] = nu[j];
        }
    }
    if (g == 0 && tid == 0) P.s_max[(int64_t)w.f * P.B + w.b] = smax;
}

// XOR of the Philox blocks [j * blocks, (j + 1) * blocks) of one sweep's
// stream, in the sweep kernels' form (two interleaved blocks per step).
__global__ void philox_xor_kernel(uint32_t key0, uint32_t key1, uint64_t t, uint32_t chain, uint32_t phase,
                                  int64_t blocks, int64_t n_out, uint32_t *__restrict__ out) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n_out) return;
    const Key2 key{key0, key1};
    const PhiloxSweep ps = philox_sweep_consts((uint32_t)t, chain, (uint32_t)(t >> 32), key);
    const uint32_t first = (uint32_t)(j * blocks), ph = phase ? kPhaseVisible : kPhaseHidden;
    uint32_t acc = 0;
    int64_t i = 0;
    for (; i + 1 < blocks; i += 2) {
        uint4 r[2];
        const uint32_t w[2] = {ph | (first + (uint32_t)i), ph | (first + (uint32_t)i + 1u)};
        philox_sweep_multi<2>(r, w, ps, key);
        acc ^= r[0].x ^ r[0].y ^ r[0].z ^ r[0].w ^ r[1].x ^ r[1].y ^ r[1].z ^ r[1].w;
    }
    if (i < blocks) {
        const uint4 r = philox_sweep(ph | (first + (uint32_t)i), ps, key);
        acc ^= r.x ^ r.y ^ r.z ^ r.w;
    }
    out[j] = acc;
}

hipError_t launch_philox_xor(uint64_t seed, int32_t formula, int64_t t, int32_t chain, int32_t phase, int64_t blocks,
                             int64_t n_out, uint32_t *out, hipStream_t s) {
    const int64_t grid = (n_out + 255) / 256;
    philox_xor_kernel<<<(unsigned)grid, 256, 0, s>>>((uint32_t)seed, (uint32_t)(seed >> 32) ^ (uint32_t)formula,
                                                     (uint64_t)t, (uint32_t)chain, (uint32_t)phase, blocks, n_out,
                                                     out);
    return hipGetLastError();
}

__global__ void zero_u32_kernel(uint32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void advance_t_kernel(int64_t *t, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t[0] += n;
}

hipError_t launch_zero(uint32_t *ptr, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    zero_u32_kernel<<<blocks, 256, 0, s>>>(ptr, n);
    return hipGetLastError();
}

template <typename Real, int kTab>
const void *push_kernel_ptr_t(int vpt) {
    switch (vpt) {
        case 1: return (const void *)sweep_push_kernel<Real, 1, kTab>;
        case 2: return (const void *)sweep_push_kernel<Real, 2, kTab>;
        case 4: return (const void *)sweep_push_kernel<Real, 4, kTab>;
        default: return (const void *)sweep_push_kernel<Real, 0, kTab>;
    }
}

// variable groups per thread kept in registers: 0 (EMA in global memory), 1, 2 or 4
template <typename Real>
const void *push_kernel_ptr(int vpt, int kind) {
    return kind == kBucketWide ? push_kernel_ptr_t<Real, kBucketWide>(vpt)
           : kind == kBucketMid ? push_kernel_ptr_t<Real, kBucketMid>(vpt)
                                : push_kernel_ptr_t<Real, kBucketPush>(vpt);
}

template <typename Real>
const void *clust_kernel_ptr(int vpt) {
    switch (vpt) {
        case 1: return (const void *)sweep_push_kernel<Real, 1, kBucketPush, false, true>;
        case 2: return (const void *)sweep_push_kernel<Real, 2, kBucketPush, false, true>;
        case 4: return (const void *)sweep_push_kernel<Real, 4, kBucketPush, false, true>;
        default: return (const void *)sweep_push_kernel<Real, 0, kBucketPush, false, true>;
    }
}

// owned variables per thread of a split member: 1 or 2 in registers, else 0
template <typename Real>
const void *split_kernel_ptr(bool clust, int vpt) {
    if (clust)
        return vpt == 1 ? (const void *)sweep_split_kernel<Real, 1, true>
               : vpt == 2 ? (const void *)sweep_split_kernel<Real, 2, true>
                          : (const void *)sweep_split_kernel<Real, 0, true>;
    return vpt == 1 ? (const void *)sweep_split_kernel<Real, 1>
           : vpt == 2 ? (const void *)sweep_split_kernel<Real, 2>
                      : (const void *)sweep_split_kernel<Real, 0>;
}

const void *mixed_kernel_ptr(int vpt) {
    switch (vpt) {
        case 1: return (const void *)sweep_push_kernel<double, 1, kBucketWide, true>;
        case 2: return (const void *)sweep_push_kernel<double, 2, kBucketWide, true>;
        default: return (const void *)sweep_push_kernel<double, 0, kBucketWide, true>;
    }
}

template <typename Real>
const void *pull_kernel_ptr(int vpt) {
    switch (vpt) {
        case 1: return (const void *)sweep_pull_kernel<Real, 1>;
        case 2: return (const void *)sweep_pull_kernel<Real, 2>;
        default: return (const void *)sweep_pull_kernel<Real, 0>;
    }
}

template <typename Real>
hipError_t set_limits_t(int bytes) {
    std::vector<const void *> ks;
    for (int vpt : {0, 1, 2, 4}) {
        for (int kind : {(int)kBucketPush, (int)kBucketWide, (int)kBucketMid}) ks.push_back(push_kernel_ptr<Real>(vpt, kind));
        ks.push_back(clust_kernel_ptr<Real>(vpt));
    }
    for (int vpt : {0, 1, 2}) {
        ks.push_back(pull_kernel_ptr<Real>(vpt));
        ks.push_back(split_kernel_ptr<Real>(false, vpt));
        ks.push_back(split_kernel_ptr<Real>(true, vpt));
    }
    for (const void *k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t set_kernel_lds_limits(int bytes) {
    hipError_t e = set_limits_t<double>(bytes);
    if (e == hipSuccess) e = set_limits_t<float>(bytes);
    for (int vpt = 0; vpt < 3 && e == hipSuccess; ++vpt)
        e = hipFuncSetAttribute(mixed_kernel_ptr(vpt), hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

int bucket_occupancy(const Plan &p, const Bucket &b) {
    const void *k;
    if (b.kind == kBucketPull)
        k = p.precision == HP_FP32 ? pull_kernel_ptr<float>(b.vpt) : pull_kernel_ptr<double>(b.vpt);
    else if (p.precision == HP_MIXED_BF16)
        k = mixed_kernel_ptr(b.vpt);
    else if (p.clust)
        k = p.precision == HP_FP64 ? clust_kernel_ptr<double>(b.vpt) : clust_kernel_ptr<float>(b.vpt);
    else
        k = p.precision == HP_FP64 ? push_kernel_ptr<double>(b.vpt, b.kind) : push_kernel_ptr<float>(b.vpt, b.kind);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, b.threads, b.lds) != hipSuccess) return 1;
    return nb;
}

int split_vpt(int max_n, int G, int threads) {
    const int groups = (max_n + 3) / 4;
    const int owned = 4 * ((groups + G - 1) / G);   // variables per member
    return owned <= threads ? 1 : owned <= 2 * threads ? 2 : 0;
}

int split_occupancy(const Plan &p, int G) {
    int nb = 0;
    const Bucket &b = p.buckets[0];
    const int vpt = split_vpt(b.max_n, G, b.threads);
    const void *kern = p.precision == HP_FP64 ? split_kernel_ptr<double>(p.clust, vpt)
                                              : split_kernel_ptr<float>(p.clust, vpt);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, b.threads, b.lds) != hipSuccess) return 0;
    return nb;
}

template <typename Real>
hipError_t launch_split_one(const Plan &p, SweepParams<Real> P, SplitParams Q, int vpt, hipStream_t s) {
    const Bucket &b = p.buckets[0];
    // The plan checked that all count*G workgroups fit on the device at once
    // (occupancy x CUs), so on an otherwise idle device they are all resident
    // together; the waits for the other members are bounded either way (see hp_check).
    hipLaunchKernelGGL((void (*)(SweepParams<Real>, SplitParams))split_kernel_ptr<Real>(p.clust, vpt),
                       dim3(b.count * p.split), dim3(b.threads), b.lds, s, P, Q);
    return hipGetLastError();
}

template <typename Real>
SweepParams<Real> sweep_params(const Plan &p, const hp_state &st, int64_t n_sweeps) {
    SweepParams<Real> P;
    P.fd = p.d_fd;
    P.work = p.d_work;
    P.lits = p.d_lits;
    P.csr_ptr = p.d_csr_ptr;
    P.occ = p.d_occ;
    P.rec = p.d_rec;
    P.orig = p.d_orig;
    P.negcnt = p.d_negcnt;
    P.gfx = p.tab.gfx;
    P.gpad = p.tab.gpad;
    P.mfma = p.tab.mfma;
    P.fx_scale = std::ldexp(1.0, -p.fx_shift);
    P.thr = p.tab.thr;
    P.G = std::is_same<Real, double>::value ? reinterpret_cast<const Real *>(p.tab.g64)
                                            : reinterpret_cast<const Real *>(p.tab.g32);
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
    P.lds_v_off = P.lds_x_off = P.lds_hm_off = 0;
    P.dyn_steps = 1;
    return P;
}

// --------------------------------------------------------------------------
// Run buffers: the plan's own, or the static scratch of hp_run_noalloc
// --------------------------------------------------------------------------
// The scratch array lives in this code object; on the host its name is a
// stand-in, so kernels receive the device address that hipGetSymbolAddress
// returns for the current device (each device has its own copy).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[kMaxDevices] = {};

hipError_t static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[device]) return hipSuccess;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = ptr;
    return hipSuccess;
}

void *static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_addr[device];
}

RunBuffers plan_buffers(const Plan &p) { return RunBuffers{p.d_queue, p.d_xpart, p.d_vbuf, p.d_cnt}; }

static size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// layout: work counters | xpart | vbuf | counts, each 256-byte aligned
static void scratch_layout(const Plan &p, size_t off[4], size_t *total) {
    const size_t items = p.split > 1 ? (size_t)p.buckets[0].count : 0;
    off[0] = 0;
    off[1] = align256(off[0] + (size_t)kMaxBuckets * kQueueWords * sizeof(uint32_t));
    off[2] = align256(off[1] + items * p.split * p.nstride * sizeof(int64_t));
    off[3] = align256(off[2] + items * p.nstride);
    *total = align256(off[3] + items * 2 * kMaxSplit * sizeof(int32_t));
}

size_t run_scratch_bytes(const Plan &p) {
    size_t off[4], total = 0;
    scratch_layout(p, off, &total);
    return total;
}

RunBuffers scratch_buffers(const Plan &p, void *base) {
    size_t off[4], total = 0;
    scratch_layout(p, off, &total);
    unsigned char *b = static_cast<unsigned char *>(base);
    const bool split = p.split > 1;
    return RunBuffers{reinterpret_cast<uint32_t *>(b + off[0]), split ? reinterpret_cast<int64_t *>(b + off[1]) : nullptr,
                      split ? b + off[2] : nullptr, split ? reinterpret_cast<int32_t *>(b + off[3]) : nullptr};
}

template <typename Real>
hipError_t launch_bucket_t(const Plan &p, const Bucket &b, const hp_state &st, int64_t n_sweeps, hipStream_t s,
                           uint32_t *queues) {
    if (b.count == 0) return hipSuccess;
    SweepParams<Real> P = sweep_params<Real>(p, st, n_sweeps);
    P.work = p.d_work + b.first;
    P.lds_v_off = b.v_off;
    P.lds_x_off = b.x_off;
    P.lds_hm_off = b.hm_off;
    P.dyn_steps = b.dyn;
    if (b.kind == kBucketPull) {
        hipLaunchKernelGGL((void (*)(SweepParams<Real>))pull_kernel_ptr<Real>(b.vpt), dim3(b.count), dim3(b.threads),
                           b.lds, s, P);
        return hipGetLastError();
    }
    WorkQueue Q;
    Q.ctr = nullptr;
    Q.count = b.count;
    for (int x = 0; x <= kXcds; ++x) Q.xq[x] = b.xq[x];
    int grid = b.count;
    if (b.grid > 0) {
        // the bucket's counters: one 128-byte line per XCD
        Q.ctr = queues + kQueueWords * (size_t)(&b - p.buckets.data());
        hipError_t e = launch_zero(Q.ctr, kQueueWords, s);
        if (e != hipSuccess) return e;
        grid = b.grid;
    }
    const void *kern = p.precision == HP_MIXED_BF16 ? mixed_kernel_ptr(b.vpt)
                       : p.clust                     ? clust_kernel_ptr<Real>(b.vpt)
                                                     : push_kernel_ptr<Real>(b.vpt, b.kind);
    hipLaunchKernelGGL((void (*)(SweepParams<Real>, WorkQueue))kern, dim3(grid), dim3(b.threads), b.lds, s, P, Q);
    return hipGetLastError();
}

static hipError_t launch_bucket_q(const Plan &p, const Bucket &b, const hp_state &st, int64_t n_sweeps, hipStream_t s,
                                  uint32_t *queues) {
    return p.precision == HP_FP32 ? launch_bucket_t<float>(p, b, st, n_sweeps, s, queues)
                                  : launch_bucket_t<double>(p, b, st, n_sweeps, s, queues);
}

hipError_t launch_bucket(const Plan &p, const Bucket &b, const hp_state &st, int64_t n_sweeps, hipStream_t s) {
    return launch_bucket_q(p, b, st, n_sweeps, s, p.d_queue);
}

template <typename Real>
hipError_t launch_split_t(const Plan &p, const hp_state &st, int64_t n_sweeps, hipStream_t s, const RunBuffers &rb) {
    const Bucket &b = p.buckets[0];
    SweepParams<Real> P = sweep_params<Real>(p, st, n_sweeps);
    P.lds_v_off = b.v_off;
    P.lds_x_off = b.x_off;
    SplitParams Q;
    Q.xpart = rb.xpart;
    Q.vbuf = rb.vbuf;
    Q.cnt = rb.cnt;
    Q.err = p.d_err;
    Q.nstride = p.nstride;
    Q.G = p.split;
    Q.wait_limit = p.wait_limit > 0 ? (uint32_t)p.wait_limit : kMailSpins;
    Q.xcd_map = p.xcd_map;
    Q.n_xcd = 8;
    // every mailbox starts with tag 0 (no sweep's tag)
    hipError_t e = launch_zero(reinterpret_cast<uint32_t *>(rb.xpart), (int64_t)b.count * p.split * p.nstride * 2, s);
    if (e == hipSuccess) e = launch_zero(reinterpret_cast<uint32_t *>(rb.vbuf), (int64_t)b.count * p.nstride / 4, s);
    if (e == hipSuccess) e = launch_zero(reinterpret_cast<uint32_t *>(rb.cnt), (int64_t)b.count * 2 * kMaxSplit, s);
    if (e != hipSuccess) return e;
    return launch_split_one<Real>(p, P, Q, split_vpt(b.max_n, p.split, b.threads), s);
}

// All launches of one run: a split launch, one bucket on the caller's
// stream, or several buckets (they are independent) either forked onto side
// streams and joined back, so that one bucket's tail overlaps the next, or in
// sequence on the caller's stream (each persistent grid fills the GPU by
// itself; the autotuner keeps the faster order); then the sweep counter
// advances.
hipError_t launch_sweep(const Plan &p, const hp_state &st, int64_t n_sweeps, hipStream_t s) {
    return launch_sweep(p, st, n_sweeps, s, plan_buffers(p));
}

hipError_t launch_buckets(const Plan &p, const hp_state &st, int64_t n_sweeps, hipStream_t s, const RunBuffers &rb) {
    hipError_t e = hipSuccess;
    if (p.split > 1) {
        e = p.precision == HP_FP64 ? launch_split_t<double>(p, st, n_sweeps, s, rb)
                                   : launch_split_t<float>(p, st, n_sweeps, s, rb);
    } else if (p.buckets.size() == 1 || !p.forked) {
        for (size_t i = 0; i < p.buckets.size() && e == hipSuccess; ++i)
            e = launch_bucket_q(p, p.buckets[i], st, n_sweeps, s, rb.queue);
    } else {
        e = hipEventRecord(p.ev_fork, s);
        for (size_t i = 0; i < p.buckets.size() && e == hipSuccess; ++i) {
            e = hipStreamWaitEvent(p.side[i], p.ev_fork, 0);
            if (e == hipSuccess) e = launch_bucket_q(p, p.buckets[i], st, n_sweeps, p.side[i], rb.queue);
            if (e == hipSuccess) e = hipEventRecord(p.ev_join[i], p.side[i]);
        }
        for (size_t i = 0; i < p.buckets.size() && e == hipSuccess; ++i) e = hipStreamWaitEvent(s, p.ev_join[i], 0);
    }
    return e;
}

hipError_t launch_sweep(const Plan &p, const hp_state &st, int64_t n_sweeps, hipStream_t s, const RunBuffers &rb) {
    hipError_t e = launch_buckets(p, st, n_sweeps, s, rb);
    if (e != hipSuccess) return e;
    if (n_sweeps > 0) {
        advance_t_kernel<<<1, 64, 0, s>>>(st.t, n_sweeps);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace hp
