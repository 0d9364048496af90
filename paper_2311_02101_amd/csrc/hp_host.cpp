// C-ABI entry points: validation, formula-RBM assembly (packing of the clause
// table and the per-variable occurrence lists), device allocation and launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "hp_internal.hpp"

namespace hp {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

hp_status fail(hp_status s, const std::string &msg) {
    set_error(msg);
    return s;
}

hp_status hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? HP_ENOMEM : HP_EDEVICE;
}

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src, hipStream_t s) {
    *dst = nullptr;
    if (src.empty()) return hipSuccess;
    hipError_t e = hipMalloc((void **)dst, src.size() * sizeof(T));
    if (e != hipSuccess) return e;
    // src is kept alive by the caller until the copy completes (synchronised
    // at the end of hp_plan), so an asynchronous copy is safe
    return hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

void release(Plan *p) {
    if (!p) return;
    for (GraphEntry &g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    for (int i = 0; i < kMaxBuckets; ++i) {
        if (p->side[i]) (void)hipStreamDestroy(p->side[i]);
        if (p->ev_join[i]) (void)hipEventDestroy(p->ev_join[i]);
    }
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    (void)hipFree(p->d_queue);
    (void)hipFree(p->d_var_off);
    (void)hipFree(p->d_clause_off);
    (void)hipFree(p->d_feat_acc);
    (void)hipFree(p->d_fd);
    (void)hipFree(p->d_work);
    (void)hipFree(p->d_work_fb);
    (void)hipFree(p->d_mg_cnt);
    (void)hipFree(p->d_mg_v);
    (void)hipFree(p->d_mg_nu);
    (void)hipFree(p->d_lits);
    (void)hipFree(p->d_csr_ptr);
    (void)hipFree(p->d_occ);
    (void)hipFree(p->d_rec);
    (void)hipFree(p->d_orig);
    (void)hipFree(p->d_negcnt);
    (void)hipFree(p->d_tabflag);
    (void)hipFree(p->tab.gfx);
    (void)hipFree(p->tab.gpad);
    (void)hipFree(p->d_xpart);
    (void)hipFree(p->d_vbuf);
    (void)hipFree(p->d_cnt);
    (void)hipFree(p->d_err);
    (void)hipFree(p->d_temp);
    (void)hipFree(p->d_fe);
    (void)hipFree(p->d_fe_chain);
    (void)hipFree(p->d_temp_old);
    (void)hipFree(p->d_W);
    (void)hipFree(p->d_b);
    (void)hipFree(p->d_Wc);
    (void)hipFree(p->d_bc);
    (void)hipFree(p->tab.thr);
    (void)hipFree(p->tab.g64);
    (void)hipFree(p->tab.g32);
    (void)hipFree(p->tab.mfma);
    delete p;
}


// Variable groups (of 4) per thread whose variance EMA stays in registers:
// 1, 2 (FP32 and FP64) or 4 (FP32), else 0 (EMA in global memory).  The
// mixed-precision kernel keeps at most one group in registers (two spill
// next to its MFMA operands); four FP64 groups spill.
int vpt_for(int groups, int threads, bool mixed, bool fp64) {
    if (groups <= threads) return 1;
    if (groups <= 2 * threads && !mixed) return 2;
    if (groups <= 4 * threads && !mixed && !fp64) return 4;
    return 0;
}

// Split a column of 8 weights into kLimbs BF16 limbs on the column's common
// exponent grid (see the mixed-precision operand layout): limb j of entry i
// is q * 2^(E - 8(j+1)) with |q| <= 256, rounded to nearest from what the
// earlier limbs left.  Returns false if a limb is not exactly a BF16 value.
bool split_limbs(const double col[8], double limb[kLimbs][8]) {
    double mx = 0.0;
    for (int i = 0; i < 8; ++i) mx = std::max(mx, std::fabs(col[i]));
    for (int j = 0; j < kLimbs; ++j)
        for (int i = 0; i < 8; ++i) limb[j][i] = 0.0;
    if (mx == 0.0) return true;
    int E = 0;
    (void)std::frexp(mx, &E);          // mx < 2^E
    double r[8];
    for (int i = 0; i < 8; ++i) r[i] = col[i];
    for (int j = 0; j < kLimbs; ++j) {
        const double grid = std::ldexp(1.0, E - 8 * (j + 1));
        for (int i = 0; i < 8; ++i) {
            const double q = std::nearbyint(r[i] / grid);
            if (std::fabs(q) > 256.0) return false;
            limb[j][i] = q * grid;
            r[i] -= limb[j][i];
            const float f = (float)limb[j][i];
            uint32_t bits;
            std::memcpy(&bits, &f, 4);
            if ((double)f != limb[j][i] || (bits & 0xffffu) != 0u) return false;
        }
    }
    return true;
}

uint16_t bf16_bits_exact(double x) {
    const float f = (float)x;
    uint32_t bits;
    std::memcpy(&bits, &f, 4);
    return (uint16_t)(bits >> 16);
}

// Per-lane A operands of the two mixed-precision products for every
// temperature: [T][2][64] uint4 (8 BF16 values each).  Lane l supplies row
// l % 32 = 8g + (unit or slot) and K entries 8h .. 8h+7 with h = l / 32, i.e.
// limb 2g + h of the 8 weights of that row.
bool mfma_operands(const double *W, const double *b, int T, int K, int L, std::vector<uint4> &out) {
    out.assign((size_t)T * 2 * 64, make_uint4(0, 0, 0, 0));
    for (int tau = 0; tau < T; ++tau) {
        const double *Wt = W + (size_t)tau * K * L;
        // product 1: column u = (W[0..K-1][u], 0.., b[u] at position 7)
        for (int u = 0; u < kMaxL; ++u) {
            double col[8] = {0, 0, 0, 0, 0, 0, 0, 0}, limb[kLimbs][8];
            if (u < L) {
                for (int k = 0; k < K; ++k) col[k] = Wt[k * L + u];
                col[7] = b[(size_t)tau * L + u];
            }
            if (!split_limbs(col, limb)) return false;
            for (int g = 0; g < kLimbs / 2; ++g)
                for (int h = 0; h < 2; ++h) {
                    uint16_t e[8];
                    for (int k = 0; k < 8; ++k) e[k] = bf16_bits_exact(limb[2 * g + h][k]);
                    out[((size_t)tau * 2 + 0) * 64 + h * 32 + g * 8 + u] =
                        make_uint4(e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16),
                                   e[4] | ((uint32_t)e[5] << 16), e[6] | ((uint32_t)e[7] << 16));
                }
        }
        // product 2: column k = (W[k][0..L-1])
        for (int k = 0; k < kMaxL; ++k) {
            double col[8] = {0, 0, 0, 0, 0, 0, 0, 0}, limb[kLimbs][8];
            if (k < K)
                for (int u = 0; u < L; ++u) col[u] = Wt[k * L + u];
            if (!split_limbs(col, limb)) return false;
            for (int g = 0; g < kLimbs / 2; ++g)
                for (int h = 0; h < 2; ++h) {
                    uint16_t e[8];
                    for (int u = 0; u < 8; ++u) e[u] = bf16_bits_exact(limb[2 * g + h][u]);
                    out[((size_t)tau * 2 + 1) * 64 + h * 32 + g * 8 + k] =
                        make_uint4(e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16),
                                   e[4] | ((uint32_t)e[5] << 16), e[6] | ((uint32_t)e[7] << 16));
                }
        }
    }
    return true;
}

}  // namespace
}  // namespace hp

using namespace hp;

extern "C" {

const char *hp_status_string(hp_status s) {
    switch (s) {
        case HP_OK: return "HP_OK";
        case HP_EINVAL: return "HP_EINVAL: invalid argument";
        case HP_ENOMEM: return "HP_ENOMEM: device allocation failed";
        case HP_EDEVICE: return "HP_EDEVICE: HIP runtime error";
        case HP_EUNSUPPORTED: return "HP_EUNSUPPORTED: outside what the library handles";
    }
    return "unknown hp_status";
}

const char *hp_last_error(void) { return g_last_error.c_str(); }

// Launch order of a run of several buckets.  Each persistent grid fills the
// GPU by itself, and when every launch is one they run best in sequence on
// the caller's stream (1885 against 1920 ms for the 500-sweep run of the
// 1024-formula batch: kernels resident side by side compete for the CUs);
// a launch of one workgroup per item may leave CUs free, and then the
// launches are forked over side streams to run side by side.  (Timing the
// two orders on the autotuner's short trials favours forking, which hides
// the per-item setup that dominates a run of a few sweeps.)
static void choose_order(Plan *p) {
    p->forked = 0;
    for (const Bucket &b : p->buckets)
        if (b.grid == 0) p->forked = 1;
}

hp_status hp_plan(hp_plan_t *out, const hp_cnf *cnf, const hp_rbm *rbm, const hp_opts *opts,
                  void *stream) {
    g_last_error.clear();
    if (!out || !cnf || !rbm || !opts) return fail(HP_EINVAL, "null argument");
    *out = nullptr;
    const int F = cnf->n_formulas;
    const int K = cnf->k;
    if (F < 1) return fail(HP_EINVAL, "n_formulas must be >= 1");
    if (K < 1 || K > kMaxK) return fail(HP_EINVAL, "K must be in 1..7");
    if (rbm->k != K) return fail(HP_EINVAL, "rbm.k must equal cnf.k");
    const int L = rbm->l;
    if (L < 1 || L > kMaxL) return fail(HP_EINVAL, "L must be in 1..8");
    const int T = rbm->n_temps;
    if (T < 1) return fail(HP_EINVAL, "n_temps must be >= 1");
    if (!cnf->var_offset || !cnf->clause_offset || !cnf->lits || !rbm->W || !rbm->b)
        return fail(HP_EINVAL, "null array");
    const int B = opts->chains;
    if (B < 1) return fail(HP_EINVAL, "chains must be >= 1");
    if (!(opts->alpha >= 0.0 && opts->alpha <= 1.0)) return fail(HP_EINVAL, "alpha must be in [0,1]");
    if (opts->precision != HP_FP64 && opts->precision != HP_FP32 && opts->precision != HP_MIXED_BF16)
        return fail(HP_EINVAL, "unknown precision");
    if (opts->precision == HP_MIXED_BF16 && (opts->kernel == HP_KERNEL_PULL || opts->split >= 2))
        return fail(HP_EUNSUPPORTED, "mixed BF16 precision runs the push launch without split only");
    if (opts->threads != 0 && (opts->threads < kWave || opts->threads > 1024 || opts->threads % kWave))
        return fail(HP_EINVAL, "threads must be 0 or a multiple of 64 in [64, 1024]");
    if (opts->kernel < HP_KERNEL_AUTO || opts->kernel > HP_KERNEL_PUSH)
        return fail(HP_EINVAL, "unknown kernel variant");
    if (opts->split < 0 || opts->split > kMaxSplit || (opts->split & (opts->split - 1)))
        return fail(HP_EINVAL, "split must be 0 (automatic) or a power of two up to 16");
    if (opts->graph && opts->split > 1) return fail(HP_EINVAL, "graph mode does not capture split launches");
    if (opts->split_wait_limit < 0) return fail(HP_EINVAL, "split_wait_limit must be >= 0");
    for (int i = 0; i < T * K * L; ++i)
        if (!std::isfinite(rbm->W[i])) return fail(HP_EINVAL, "non-finite weight");
    for (int i = 0; i < T * L; ++i)
        if (!std::isfinite(rbm->b[i])) return fail(HP_EINVAL, "non-finite bias");
    // size-clustered model: the RBMs of the groups K = 3 .. max(K, 3)
    const bool clust = opts->size_rbms != nullptr;
    const int n_groups = clust ? std::max(K, 3) - 2 : 0;
    if (clust) {
        if (opts->precision == HP_MIXED_BF16 || opts->kernel == HP_KERNEL_PULL)
            return fail(HP_EUNSUPPORTED, "the size-clustered model runs the push launch in FP64 or FP32 only");
        for (int i = 0; i < n_groups; ++i) {
            const hp_rbm &r = opts->size_rbms[i];
            const int Kg = 3 + i;
            if (r.k != Kg || r.l != clust_hidden(Kg) || r.n_temps != T || !r.W || !r.b)
                return fail(HP_EINVAL, "size_rbms[" + std::to_string(i) + "] must be the K = " + std::to_string(Kg) +
                                           " RBM with L = " + std::to_string(clust_hidden(Kg)) +
                                           " and the plan's n_temps");
            for (int j = 0; j < T * Kg * r.l; ++j)
                if (!std::isfinite(r.W[j])) return fail(HP_EINVAL, "non-finite weight in size_rbms");
            for (int j = 0; j < T * r.l; ++j)
                if (!std::isfinite(r.b[j])) return fail(HP_EINVAL, "non-finite bias in size_rbms");
        }
    }
    // temperature of every (formula, chain); replica exchange changes them per formula
    std::vector<int32_t> temp((size_t)F * B);
    for (int b = 0; b < B; ++b) {
        const int32_t t = opts->temp_of_chain ? opts->temp_of_chain[b] : (int32_t)((int64_t)b * T / B);
        if (t < 0 || t >= T) return fail(HP_EINVAL, "temperature index out of range");
        for (int f = 0; f < F; ++f) temp[(size_t)f * B + b] = t;
    }
    if (cnf->var_offset[0] != 0 || cnf->clause_offset[0] != 0)
        return fail(HP_EINVAL, "offsets must start at 0");
    int max_n = 0, max_c = 0;
    for (int f = 0; f < F; ++f) {
        const int64_t n = cnf->var_offset[f + 1] - cnf->var_offset[f];
        const int64_t c = cnf->clause_offset[f + 1] - cnf->clause_offset[f];
        if (n < 1 || c < 1) return fail(HP_EINVAL, "every formula needs N_f >= 1 and C_f >= 1");
        if (n > kMaxVars) return fail(HP_EUNSUPPORTED, "N_f above 32768");
        if (c >= (int64_t(1) << 28)) return fail(HP_EUNSUPPORTED, "C_f too large");
        max_n = std::max<int>(max_n, (int)n);
        max_c = std::max<int>(max_c, (int)c);
    }
    const int64_t NV = cnf->var_offset[F], NC = cnf->clause_offset[F];
    if ((int64_t)K * NC >= (int64_t(1) << 32)) return fail(HP_EUNSUPPORTED, "too many clause slots");

    // --- per formula (independent, so formulas are packed on host threads):
    //   clause table: padding normalisation + packing (idx | neg << 15);
    //   per-variable occurrence lists, (c, k) ascending (formula f's lists
    //   start at K * clause_offset[f]: every clause has K slots);
    //   push-kernel clause records: length, padding merge, sort by length.
    //   len = K minus the trailing run of copies of literal 0 (the padding of
    //   Sec. 3.3); positions >= len contribute through the merged slot 0.
    std::vector<uint16_t> lits((size_t)K * NC);
    std::vector<uint32_t> deg(NV, 0);
    std::vector<uint32_t> csr_ptr(NV + F);
    std::vector<uint32_t> occ((size_t)K * NC);
    std::vector<uint4> rec(NC);
    // orig[]: the first Philox block of each record's hidden draw (the
    // clause's input index times its blocks per clause, two in the
    // size-clustered model), so the kernels add the unit's block offset only
    const uint32_t blocks_per_clause = clust ? 2u : (uint32_t)(L + 3) / 4u;
    if ((int64_t)max_c * blocks_per_clause > (int64_t(1) << 31))
        return fail(HP_EUNSUPPORTED, "a formula's hidden draws would need more than 2^31 Philox blocks per sweep");
    std::vector<uint32_t> orig(NC);
    std::vector<uint32_t> push_slots(NV, 0);
    std::vector<int32_t> negcnt(NV, 0);
    std::vector<std::array<int32_t, 8>> lofs(F);
    std::vector<std::string> pack_err(F);
    auto pack_formula = [&](int f) -> std::string {
        const int64_t v0 = cnf->var_offset[f], n = cnf->var_offset[f + 1] - v0;
        const int64_t c0 = cnf->clause_offset[f], c1 = cnf->clause_offset[f + 1];
        for (int64_t c = c0; c < c1; ++c) {
            int32_t first = 0;
            for (int k = 0; k < K; ++k)
                if (cnf->lits[(size_t)k * NC + c] != 0) {
                    first = cnf->lits[(size_t)k * NC + c];
                    break;
                }
            if (first == 0) return "clause " + std::to_string(c) + " has no literal";
            for (int k = 0; k < K; ++k) {
                int32_t x = cnf->lits[(size_t)k * NC + c];
                if (x == 0) x = first;
                const int64_t a = x < 0 ? -(int64_t)x : (int64_t)x;
                if (a > n) return "literal " + std::to_string(x) + " exceeds N_f";
                lits[(size_t)k * NC + c] = (uint16_t)((a - 1) | (x < 0 ? 0x8000u : 0u));
                deg[v0 + a - 1]++;
            }
        }
        uint64_t pos = (uint64_t)K * (uint64_t)c0;
        for (int64_t i = 0; i < n; ++i) {
            csr_ptr[v0 + f + i] = (uint32_t)pos;
            pos += deg[v0 + i];
        }
        csr_ptr[v0 + f + n] = (uint32_t)pos;
        std::vector<uint32_t> fill(csr_ptr.begin() + v0 + f, csr_ptr.begin() + v0 + f + n);
        for (int64_t c = c0; c < c1; ++c)
            for (int k = 0; k < K; ++k) {
                const uint16_t e = lits[(size_t)k * NC + c];
                occ[fill[e & 0x7fff]++] = ((uint32_t)(c - c0) << 4) | ((e >> 15) << 3) | (uint32_t)k;
            }
        std::vector<std::pair<int, int64_t>> key;
        key.reserve(c1 - c0);
        for (int64_t c = c0; c < c1; ++c) {
            int len = K;
            while (len > 1 && lits[(size_t)(len - 1) * NC + c] == lits[c]) --len;
            key.push_back({len, c});
            for (int k = 0; k < len; ++k) {
                const uint16_t e = lits[(size_t)k * NC + c];
                push_slots[v0 + (e & 0x7fff)]++;
                if (e >> 15) negcnt[v0 + (e & 0x7fff)]++;
            }
        }
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<int, int64_t> &a, const std::pair<int, int64_t> &b) {
                             return a.first < b.first;
                         });
        // records of length <= k: the bounds of the kernels' per-length runs
        lofs[f].fill(0);
        for (const auto &kc : key)
            for (int k = kc.first; k < 8; ++k) lofs[f][k]++;
        for (int64_t j = 0; j < c1 - c0; ++j) {
            const int len = key[j].first;
            const int64_t c = key[j].second;
            uint16_t sl[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            uint32_t negm = 0;
            for (int k = 0; k < K; ++k) sl[k] = lits[(size_t)k * NC + c];
            for (int k = 0; k < len; ++k) negm |= (uint32_t)(sl[k] >> 15) << k;
            // below seven literals the last word is the negation bits | 2^len
            // alone (its XOR with the literals' values is the push kernels'
            // threshold row 2^len + pattern); seven literals keep slot 6 and
            // len | negm << 3 above it
            if (len < 7) {
                sl[6] = (uint16_t)(negm | (1u << len));
                sl[7] = 0;
            } else {
                sl[7] = (uint16_t)(len | (negm << 3));
            }
            rec[c0 + j] = make_uint4(sl[0] | ((uint32_t)sl[1] << 16), sl[2] | ((uint32_t)sl[3] << 16),
                                     sl[4] | ((uint32_t)sl[5] << 16), sl[6] | ((uint32_t)sl[7] << 16));
            orig[c0 + j] = (uint32_t)(c - c0) * blocks_per_clause;
        }
        return std::string();
    };
    {
        // contiguous runs of formulas of about equal clause counts per thread
        int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
        if (F < 2 || NC < (int64_t(1) << 16)) nt = 1;
        nt = std::min(nt, F);
        std::vector<int> first(nt + 1, F);
        first[0] = 0;
        for (int t = 1, f = 0; t < nt; ++t) {
            const int64_t target = NC * t / nt;
            while (f < F && cnf->clause_offset[f] < target) ++f;
            first[t] = f;
        }
        auto run = [&](int t) {
            for (int f = first[t]; f < first[t + 1]; ++f) pack_err[f] = pack_formula(f);
        };
        if (nt == 1) {
            run(0);
        } else {
            std::vector<std::thread> pool;
            for (int t = 0; t < nt; ++t) pool.emplace_back(run, t);
            for (std::thread &th : pool) th.join();
        }
        for (int f = 0; f < F; ++f)
            if (!pack_err[f].empty()) return fail(HP_EINVAL, pack_err[f]);
    }
    // fixed-point scale: every slot contributes at most Wsum = sum |W_c| in
    // magnitude, a variable has at most max_slots slots, so |x| * 2^S stays
    // below 2^61 when (bound + 1) * 2^S < 2^61 (the split exchange tags bits
    // 61 and 62 of a partial sum, which needs bits 61..63 to be sign copies)
    double wsum = 0.0;
    for (int t = 0; t < T; ++t) {
        if (clust) {
            for (int i = 0; i < n_groups; ++i) {
                const int KL = (3 + i) * opts->size_rbms[i].l;
                double s = 0.0;
                for (int j = 0; j < KL; ++j) s += std::fabs(opts->size_rbms[i].W[(size_t)t * KL + j]);
                wsum = std::max(wsum, s);
            }
            continue;
        }
        double s = 0.0;
        for (int i = 0; i < K * L; ++i) s += std::fabs(rbm->W[(size_t)t * K * L + i]);
        wsum = std::max(wsum, s);
    }
    uint32_t max_slots = 1;
    for (int64_t i = 0; i < NV; ++i) max_slots = std::max(max_slots, push_slots[i]);
    const double bound = wsum * (double)max_slots * (1.0 + 1e-9) + 8.0;
    int fx_shift = 52;
    while (fx_shift > 0 && std::ldexp(bound + 1.0, fx_shift) >= std::ldexp(1.0, 61)) --fx_shift;

    // --- formula descriptors ---
    std::vector<FormulaDev> fd(F);
    for (int f = 0; f < F; ++f) {
        fd[f].n = (int32_t)(cnf->var_offset[f + 1] - cnf->var_offset[f]);
        fd[f].c = (int32_t)(cnf->clause_offset[f + 1] - cnf->clause_offset[f]);
        fd[f].var_off = cnf->var_offset[f];
        fd[f].clause_off = cnf->clause_offset[f];
        fd[f].ptr_off = cnf->var_offset[f] + f;
        for (int k = 0; k < 8; ++k) fd[f].lofs[k] = lofs[f][k];
    }

    Plan *p = new (std::nothrow) Plan();
    if (!p) return fail(HP_ENOMEM, "host allocation failed");
    p->F = F; p->K = K; p->L = L; p->T = T; p->B = B;
    p->precision = opts->precision;
    p->alpha = opts->alpha;
    p->seed = opts->seed;
    p->total_vars = NV; p->total_clauses = NC; p->total_occ = (int64_t)K * NC;
    p->max_n = max_n; p->max_c = max_c;
    p->fx_shift = fx_shift;
    p->clust = clust ? 1 : 0;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { release(p); return hip_fail(e, "hipGetDevice"); }
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
    if (e != hipSuccess) { release(p); return hip_fail(e, "hipDeviceGetAttribute"); }
    const size_t real_bytes = opts->precision == HP_FP32 ? 4 : 8;
    const bool mixed = opts->precision == HP_MIXED_BF16;
    p->threads = opts->threads;

    // --- kernel variant and size class per formula, work list, buckets ---
    // kind: push (tables in LDS) when everything fits, else push with the
    // merged paddings (mid) or all contribution rows (wide) in global
    // memory, else the pull kernel.  Formulas are ordered by (push or pull,
    // size class) and, inside a class, largest first; each such run of work
    // items becomes one launch.
    auto kind_of = [&](int f) -> int {
        int32_t vo, xo, ho;
        const bool fx_ok = fx_shift >= 40;
        if (mixed)   // contributions come from MFMA: only the threshold table in LDS
            return fx_ok && lds_bytes_push(fd[f].n, kBucketWide, &vo, &xo) <= (size_t)max_lds ? kBucketWide : -1;
        if (clust)   // clustered tables in LDS only
            return fx_ok && lds_bytes_clust(fd[f].n, &vo, &xo) <= (size_t)max_lds ? kBucketPush : -1;
        if (opts->kernel != HP_KERNEL_PULL && fx_ok) {
            if (lds_bytes_push(fd[f].n, kBucketPush, &vo, &xo) <= (size_t)max_lds) return kBucketPush;
            if (lds_bytes_push(fd[f].n, kBucketMid, &vo, &xo) <= (size_t)max_lds) return kBucketMid;
            if (lds_bytes_push(fd[f].n, kBucketWide, &vo, &xo) <= (size_t)max_lds) return kBucketWide;
        }
        if (opts->kernel == HP_KERNEL_PUSH) return -1;
        if (lds_bytes_pull(fd[f].n, fd[f].c, real_bytes, &vo, &ho) <= (size_t)max_lds) return kBucketPull;
        return -1;
    };
    auto size_class = [&](int f) {
        int c = 0;
        while (c < 9 && (64 << (c + 1)) <= fd[f].n) ++c;
        return c;
    };
    std::vector<int> kind(F), cls(F);
    for (int f = 0; f < F; ++f) {
        kind[f] = kind_of(f);
        if (kind[f] < 0) {
            release(p);
            if (fx_shift < 40 && (mixed || clust || opts->kernel == HP_KERNEL_PUSH))
                return fail(HP_EUNSUPPORTED, "the weights are too large for the push kernels' fixed-point "
                                             "accumulators (scale 2^" + std::to_string(fx_shift) + ", need 2^40)");
            return fail(HP_EUNSUPPORTED, "formula " + std::to_string(f) + " (N = " + std::to_string(fd[f].n) +
                                             ") does not fit the workgroup LDS limit (" + std::to_string(max_lds) +
                                             " B) with the requested kernel");
        }
        cls[f] = size_class(f);
    }
    // Buckets: one per size class of the push family (the formulas of a class
    // share a launch whatever table layout each would fit, so the chains of
    // its largest and smallest formulas balance over one persistent grid;
    // the bucket takes the layout its largest tables need: all in LDS, then
    // mid, then wide), and one per size class of pull formulas.
    auto pull_family = [&](int f) { return kind[f] == kBucketPull ? 1 : 0; };
    auto layout_rank = [](int k) { return k == kBucketPush ? 0 : k == kBucketMid ? 1 : 2; };
    std::vector<int> order(F);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (pull_family(a) != pull_family(b)) return pull_family(a) < pull_family(b);
        if (cls[a] != cls[b]) return cls[a] > cls[b];
        return (int64_t)fd[a].n * 7 + fd[a].c > (int64_t)fd[b].n * 7 + fd[b].c;
    });
    std::vector<WorkItem> work;
    work.reserve((size_t)F * B);
    for (size_t j = 0; j < order.size(); ++j) {
        const int f = order[j];
        if (j == 0 || pull_family(f) != pull_family(order[j - 1]) || cls[f] != cls[order[j - 1]]) {
            Bucket bk;
            bk.kind = kind[f];
            bk.first = (int32_t)work.size();
            p->buckets.push_back(bk);
        }
        Bucket &bk = p->buckets.back();
        if (layout_rank(kind[f]) > layout_rank(bk.kind)) bk.kind = kind[f];
        bk.max_n = std::max(bk.max_n, fd[f].n);
        bk.max_c = std::max(bk.max_c, fd[f].c);
        for (int b = 0; b < B; ++b) work.push_back({f, b});
        bk.count = (int32_t)work.size() - bk.first;
    }
    if ((int)p->buckets.size() > kMaxBuckets) {
        release(p);
        return fail(HP_EUNSUPPORTED, "too many size classes");
    }
    // XCD groups inside every bucket: whole formulas (their B chains stay
    // together), each given to the XCD with the least work so far in the
    // bucket's largest-first order; the bucket's items are reordered group by
    // group
    for (Bucket &bk : p->buckets) {
        std::vector<std::vector<WorkItem>> grp(kXcds);
        double load[kXcds] = {};
        for (int j = bk.first; j < bk.first + bk.count; j += B) {
            const int f = work[j].f;
            int x = 0;
            for (int y = 1; y < kXcds; ++y)
                if (load[y] < load[x]) x = y;
            load[x] += 7.0 * fd[f].n + fd[f].c;
            for (int b = 0; b < B; ++b) grp[x].push_back(work[j + b]);
        }
        int pos = bk.first;
        for (int x = 0; x < kXcds; ++x) {
            bk.xq[x] = pos - bk.first;
            for (const WorkItem &wi : grp[x]) work[pos++] = wi;
        }
        bk.xq[kXcds] = pos - bk.first;
    }
    p->n_work = (int32_t)work.size();
    e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) { release(p); return hip_fail(e, "hipDeviceGetAttribute"); }
    e = set_kernel_lds_limits(max_lds);
    if (e != hipSuccess) { release(p); return hip_fail(e, "hipFuncSetAttribute"); }
    for (Bucket &bk : p->buckets) {
        if (bk.kind == kBucketPull)
            bk.lds = lds_bytes_pull(bk.max_n, bk.max_c, real_bytes, &bk.v_off, &bk.hm_off);
        else if (clust)
            bk.lds = lds_bytes_clust(bk.max_n, &bk.v_off, &bk.x_off);
        else
            bk.lds = lds_bytes_push(bk.max_n, bk.kind, &bk.v_off, &bk.x_off);
        // default workgroup size: about six clauses per thread per sweep
        int t = opts->threads;
        if (t == 0) {
            t = 64;
            while (t < kMaxThreads && t * 6 < bk.max_c) t *= 2;
        }
        bk.threads = t;
        const int groups = (bk.max_n + 3) / 4;
        bk.vpt = vpt_for(groups, t, mixed, opts->precision != HP_FP32);
        // persistent grid when the items outnumber the resident workgroups
        const int occ = bucket_occupancy(*p, bk);
        const int64_t capacity = (int64_t)p->cus * std::max(occ, 1);
        bk.grid = (bk.kind != kBucketPull && bk.count > capacity) ? (int32_t)capacity : 0;
    }
    choose_order(p);

    // --- split: G co-resident workgroups per chain, single push bucket only ---
    int G = 1;
    const bool single_push = p->buckets.size() == 1 && p->buckets[0].kind == kBucketPush;
    if (opts->split >= 2 && !single_push) {
        release(p);
        return fail(HP_EUNSUPPORTED, "split needs a batch whose formulas all share one push launch");
    }
    if (single_push && opts->split != 1 && !opts->graph) {
        Bucket &bk = p->buckets[0];
        const int saved = bk.threads;
        if (opts->threads == 0) bk.threads = kMaxThreads;
        // resident workgroups of the variant a split of G members launches
        auto capacity = [&](int G) { return (int64_t)p->cus * split_occupancy(*p, G); };
        const int n_items = bk.count;
        // every member owns at least one group of 4 variables
        int min_groups = INT32_MAX;
        for (int f = 0; f < F; ++f) min_groups = std::min(min_groups, (fd[f].n + 3) / 4);
        if (opts->split >= 2) {
            G = opts->split;
            if (G > min_groups) {
                release(p);
                return fail(HP_EUNSUPPORTED, "split " + std::to_string(G) + " needs more than " +
                                                 std::to_string(4 * (G - 1)) + " variables in every formula");
            }
            if ((int64_t)n_items * G > capacity(G)) {
                release(p);
                return fail(HP_EUNSUPPORTED, "split " + std::to_string(G) + ": " +
                                                 std::to_string((int64_t)n_items * G) +
                                                 " workgroups cannot all be resident (capacity " +
                                                 std::to_string(capacity(G)) + ")");
            }
        } else {
            // largest power of two that keeps every workgroup resident and
            // leaves each member at least 1024 clauses
            while (G * 2 <= kMaxSplit && G * 2 <= min_groups && (int64_t)n_items * G * 2 <= capacity(G * 2) &&
                   bk.max_c / (G * 2) >= 1024)
                G *= 2;
        }
        if (G == 1) bk.threads = saved;   // no split: keep the bucket's own shape
        else bk.grid = 0;                 // split launches run one item per group
    }
    p->split = G;
    p->wait_limit = opts->split_wait_limit;
    if (G > 1) {
        // member-major record order: member g of a split chain takes every
        // G-th record of the length-sorted order (the same length mix for
        // every member), stored contiguously so its loads are unit-stride;
        // member g's run starts at g floor(C/G) + min(g, C mod G)
        std::vector<uint4> r2(NC);
        std::vector<uint32_t> o2(NC);
        for (int f = 0; f < F; ++f) {
            const int64_t c0 = cnf->clause_offset[f], C = cnf->clause_offset[f + 1] - c0;
            const int64_t q = C / G, rem = C % G;
            for (int64_t j = 0; j < C; ++j) {
                const int64_t g = j % G, pos = g * q + std::min<int64_t>(g, rem) + j / G;
                r2[c0 + pos] = rec[c0 + j];
                o2[c0 + pos] = orig[c0 + j];
            }
        }
        rec.swap(r2);
        orig.swap(o2);
    }
    p->nstride = ((int64_t)p->buckets[0].max_n + 127) / 128 * 128;   // 128-byte lines per item
    p->xcd_map = (p->buckets[0].count % 8 == 0) ? 1 : 0;
    p->use_graph = opts->graph ? 1 : 0;

    // --- device upload ---
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> Wv(rbm->W, rbm->W + (size_t)T * K * L), bv(rbm->b, rbm->b + (size_t)T * L);
#define HP_TRY(expr, what)                                  \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) {                             \
            (void)hipStreamSynchronize(s);                  \
            release(p);                                     \
            return hip_fail(e_, what);                      \
        }                                                   \
    } while (0)
    HP_TRY(upload(&p->d_fd, fd, s), "upload formulas");
    HP_TRY(upload(&p->d_work, work, s), "upload work list");
    std::vector<WorkItem> work_fb((size_t)F * B);
    for (int f = 0; f < F; ++f)
        for (int b = 0; b < B; ++b) work_fb[(size_t)f * B + b] = {f, b};
    HP_TRY(upload(&p->d_work_fb, work_fb, s), "upload work list (formula order)");
    HP_TRY(upload(&p->d_lits, lits, s), "upload clause table");
    HP_TRY(upload(&p->d_csr_ptr, csr_ptr, s), "upload occurrence offsets");
    HP_TRY(upload(&p->d_occ, occ, s), "upload occurrences");
    // one step of zero records past the last formula's: a wave's last step of
    // a length run loads all 64 lanes' records (the lanes past the run are
    // masked), and the step's offset travels in the loads' scalar offset,
    // which the descriptor's range check does not cover
    rec.resize((size_t)NC + kWave);
    orig.resize((size_t)NC + kWave);
    HP_TRY(upload(&p->d_rec, rec, s), "upload clause records");
    HP_TRY(upload(&p->d_orig, orig, s), "upload clause order");
    HP_TRY(upload(&p->d_negcnt, negcnt, s), "upload negation counts");
    HP_TRY(upload(&p->d_temp, temp, s), "upload temperatures");
    std::vector<int64_t> voff(cnf->var_offset, cnf->var_offset + F + 1);
    std::vector<int64_t> coff(cnf->clause_offset, cnf->clause_offset + F + 1);
    HP_TRY(upload(&p->d_var_off, voff, s), "upload variable offsets");
    HP_TRY(upload(&p->d_clause_off, coff, s), "upload clause offsets");
    HP_TRY(upload(&p->d_W, Wv, s), "upload W_c");
    HP_TRY(upload(&p->d_b, bv, s), "upload b_c");
    if (clust) {
        // the size RBMs back to back; thr / gfx / gpad in the clustered layout
        std::vector<double> Wc, bc;
        std::vector<size_t> wo(n_groups), bo(n_groups);
        for (int i = 0; i < n_groups; ++i) {
            const hp_rbm &r = opts->size_rbms[i];
            wo[i] = Wc.size();
            bo[i] = bc.size();
            Wc.insert(Wc.end(), r.W, r.W + (size_t)T * r.k * r.l);
            bc.insert(bc.end(), r.b, r.b + (size_t)T * r.l);
        }
        HP_TRY(upload(&p->d_Wc, Wc, s), "upload size RBM weights");
        HP_TRY(upload(&p->d_bc, bc, s), "upload size RBM biases");
        for (int i = 0; i < n_groups; ++i) {
            p->crbm.W[i] = p->d_Wc + wo[i];
            p->crbm.b[i] = p->d_bc + bo[i];
        }
        HP_TRY(hipMalloc((void **)&p->tab.thr, (size_t)T * kClustThrRows * kMaxL * sizeof(uint32_t)), "alloc thr");
        HP_TRY(hipMalloc((void **)&p->tab.gfx, (size_t)T * kClustGfxRows * kMaxL * sizeof(int64_t)), "alloc gfx");
        HP_TRY(hipMalloc((void **)&p->tab.gpad, (size_t)T * kClustGpad * sizeof(int64_t)), "alloc gpad");
    } else {
        HP_TRY(hipMalloc((void **)&p->tab.thr, (size_t)T * kPatterns * kMaxL * sizeof(uint32_t)), "alloc thr");
        HP_TRY(hipMalloc((void **)&p->tab.g64, (size_t)T * kHidMasks * kMaxL * sizeof(double)), "alloc g64");
        HP_TRY(hipMalloc((void **)&p->tab.g32, (size_t)T * kHidMasks * kMaxL * sizeof(float)), "alloc g32");
        HP_TRY(hipMalloc((void **)&p->tab.gfx, (size_t)T * kHidMasks * kRowWords * sizeof(int64_t)), "alloc gfx");
    }
    if (mixed) {
        std::vector<uint4> ops;
        if (!mfma_operands(rbm->W, rbm->b, T, K, L, ops)) {
            (void)hipStreamSynchronize(s);
            release(p);
            return fail(HP_EUNSUPPORTED, "a weight does not split into BF16 limbs (exponent out of range)");
        }
        HP_TRY(upload(&p->tab.mfma, ops, s), "upload MFMA operands");
    }
    HP_TRY(hipMalloc((void **)&p->d_err, sizeof(int32_t)), "alloc error flag");
    HP_TRY(launch_zero(reinterpret_cast<uint32_t *>(p->d_err), 1, s), "clear error flag");
    HP_TRY(hipMalloc((void **)&p->d_tabflag, sizeof(int32_t)), "alloc table flag");
    HP_TRY(launch_zero(reinterpret_cast<uint32_t *>(p->d_tabflag), 1, s), "clear table flag");
    HP_TRY(hipMalloc((void **)&p->d_queue, kMaxBuckets * kQueueWords * sizeof(uint32_t)), "alloc work counters");
    for (size_t i = 0; i < p->buckets.size() && p->buckets.size() > 1; ++i)
        HP_TRY(hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking), "side stream");
    if (p->buckets.size() > 1) {
        HP_TRY(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming), "event");
        for (size_t i = 0; i < p->buckets.size(); ++i)
            HP_TRY(hipEventCreateWithFlags(&p->ev_join[i], hipEventDisableTiming), "event");
    }
    if (p->use_graph) HP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "capture stream");
    if (p->split > 1) {
        const size_t items = (size_t)p->buckets[0].count;
        HP_TRY(hipMalloc((void **)&p->d_xpart, items * p->split * p->nstride * sizeof(int64_t)), "alloc xpart");
        HP_TRY(hipMalloc((void **)&p->d_vbuf, items * p->nstride), "alloc vbuf");
        HP_TRY(hipMalloc((void **)&p->d_cnt, items * 2 * kMaxSplit * sizeof(int32_t)), "alloc counts");
    }
    HP_TRY(launch_tables(*p, s), "table kernel");
    // set-up of hp_run_noalloc: this device's address of the static scratch
    HP_TRY(static_scratch_init(p->device), "hipGetSymbolAddress(scratch)");
    // host staging vectors go out of scope below: wait for the copies
    HP_TRY(hipStreamSynchronize(s), "plan upload");
    int32_t tabflag = 0;
    HP_TRY(hipMemcpy(&tabflag, p->d_tabflag, sizeof(tabflag), hipMemcpyDeviceToHost), "table flag");
#undef HP_TRY
    if (tabflag) {
        release(p);
        return fail(HP_EUNSUPPORTED, "a hidden-unit probability underflows to 0 (logit below -709)");
    }
    *out = reinterpret_cast<hp_plan_t>(p);
    return HP_OK;
}

// the checks hp_run and hp_run_noalloc share
static hp_status check_run(const Plan *p, const hp_state *st, int64_t n_sweeps) {
    if (!p || !st) return fail(HP_EINVAL, "null argument");
    if (n_sweeps < 0) return fail(HP_EINVAL, "n_sweeps must be >= 0");
    if (!st->v || !st->nu || !st->s_max || !st->best || !st->t) return fail(HP_EINVAL, "null state buffer");
    if (st->total_vars != p->total_vars || st->n_formulas != p->F || st->chains != p->B)
        return fail(HP_EINVAL, "state shape does not match the plan");
    const int want = p->precision == HP_FP32 ? 4 : 8;
    if (st->nu_bytes != want) return fail(HP_EINVAL, "nu element size does not match the precision");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != p->device) return fail(HP_EINVAL, "plan was built on another device");
    return HP_OK;
}

hp_status hp_run(hp_plan_t plan, const hp_state *st, int64_t n_sweeps, void *stream) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    const hp_status chk = check_run(p, st, n_sweeps);
    if (chk != HP_OK) return chk;
    hipError_t e = hipSuccess;
    if (!p->use_graph) {
        e = launch_sweep(*p, *st, n_sweeps, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "sweep launch");
        return HP_OK;
    }
    // graph mode: capture the run's launches once per (state buffers, sweep
    // count) on a private stream, then replay the instantiated graph on the
    // caller's stream
    GraphEntry *ge = nullptr;
    for (GraphEntry &g : p->graphs)
        if (g.v == st->v && g.nu == st->nu && g.s_max == st->s_max && g.best == st->best && g.t == st->t &&
            g.n_sweeps == n_sweeps)
            ge = &g;
    if (!ge) {
        e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t le = launch_sweep(*p, *st, n_sweeps, p->cap_stream);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(p->cap_stream, &graph);
        if (le != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le != hipSuccess ? le : e, "graph capture");
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        p->graphs.push_back({st->v, st->nu, st->s_max, st->best, st->t, n_sweeps, exec});
        ge = &p->graphs.back();
    }
    e = hipGraphLaunch(ge->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return HP_OK;
}

hp_status hp_run_noalloc(hp_plan_t plan, const hp_state *st, int64_t n_sweeps, void *stream) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    const hp_status chk = check_run(p, st, n_sweeps);
    if (chk != HP_OK) return chk;
    const size_t need = run_scratch_bytes(*p);
    if (need > kScratchBytes)
        return fail(HP_EUNSUPPORTED, "this plan's run needs " + std::to_string(need) +
                                         " bytes of scratch; hp_run_noalloc holds at most " +
                                         std::to_string(kScratchBytes) + " (use hp_run)");
    void *base = static_scratch(p->device);     // resolved by hp_plan on this device
    if (!base) return fail(HP_EDEVICE, "static scratch address not resolved on this device");
    hipError_t e = launch_sweep(*p, *st, n_sweeps, (hipStream_t)stream, scratch_buffers(*p, base));
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
    return HP_OK;
}

hp_status hp_tune(hp_plan_t plan, const hp_state *st, int64_t n_sweeps, void *stream) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !st) return fail(HP_EINVAL, "null argument");
    if (n_sweeps < 1) return fail(HP_EINVAL, "n_sweeps must be >= 1");
    if (st->total_vars != p->total_vars || st->n_formulas != p->F || st->chains != p->B ||
        st->nu_bytes != (p->precision == HP_FP32 ? 4 : 8))
        return fail(HP_EINVAL, "state shape does not match the plan");
    if (p->split > 1) return HP_OK;    // the split launch keeps its full-size workgroups
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
    for (Bucket &bk : p->buckets) {
        if (e != hipSuccess) break;
        const Bucket orig = bk;
        float best_ms = -1.0f;
        Bucket best = bk;
        // the candidate shapes: the table layout of the push kernel (every
        // table in LDS; the padding table in global memory; both contribution
        // tables in global memory -- a smaller LDS footprint lets more
        // workgroups share a CU) and the workgroup size
        std::vector<int> kinds{orig.kind};
        const bool layouts = orig.kind != kBucketPull && !p->clust && p->precision != HP_MIXED_BF16;
        if (layouts) {
            kinds.clear();
            for (int k : {(int)kBucketPush, (int)kBucketMid, (int)kBucketWide}) {
                int32_t vo, xo;
                if (lds_bytes_push(orig.max_n, k, &vo, &xo) <= (size_t)max_lds) kinds.push_back(k);
            }
        }
        for (size_t ki = 0; ki < kinds.size() && e == hipSuccess; ++ki)
        for (int t = 64; t <= kMaxThreads && e == hipSuccess; t *= 2)
        for (int dyn = 0; dyn < (orig.kind != kBucketPull && p->precision != HP_MIXED_BF16 ? 2 : 1) &&
                          e == hipSuccess; ++dyn) {
            bk = orig;
            bk.threads = t;
            bk.dyn = dyn;
            if (layouts) {
                bk.kind = kinds[ki];
                bk.lds = lds_bytes_push(bk.max_n, bk.kind, &bk.v_off, &bk.x_off);
            }
            const int groups = (bk.max_n + 3) / 4;
            bk.vpt = vpt_for(groups, t, p->precision == HP_MIXED_BF16, p->precision != HP_FP32);
            const int occ = bucket_occupancy(*p, bk);
            if (occ < 1) continue;     // this shape cannot launch
            const int64_t capacity = (int64_t)p->cus * occ;
            bk.grid = (bk.kind != kBucketPull && bk.count > capacity) ? (int32_t)capacity : 0;
            // the faster of two timed runs (the first also warms the caches)
            float ms = -1.0f;
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
                e = hipEventRecord(e0, s);
                if (e == hipSuccess) e = launch_bucket(*p, bk, *st, n_sweeps, s);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float m1 = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&m1, e0, e1);
                if (e == hipSuccess && (ms < 0.0f || m1 < ms)) ms = m1;
            }
            if (e == hipSuccess && (best_ms < 0.0f || ms < best_ms)) {
                best_ms = ms;
                best = bk;
            }
        }
        bk = best_ms < 0.0f ? orig : best;
    }
    choose_order(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "hp_tune");
    for (GraphEntry &g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    p->graphs.clear();
    return HP_OK;
}

hp_status hp_plan_query(hp_plan_t plan, hp_plan_info *out) {
    g_last_error.clear();
    const Plan *p = reinterpret_cast<const Plan *>(plan);
    if (!p || !out) return fail(HP_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->split = p->split;
    out->fx_shift = p->fx_shift;
    out->n_buckets = (int32_t)p->buckets.size();
    for (size_t i = 0; i < p->buckets.size(); ++i) {
        const Bucket &b = p->buckets[i];
        (b.kind == kBucketPull ? out->pull_items : out->push_items) += b.count;
        if (b.kind == kBucketPull) out->lds_pull = std::max<int64_t>(out->lds_pull, (int64_t)b.lds);
        else out->lds_push = std::max<int64_t>(out->lds_push, (int64_t)b.lds);
        out->threads = std::max(out->threads, b.threads);
        if (i < 16) {
            out->bucket_kind[i] = b.kind;
            out->bucket_items[i] = b.count;
            out->bucket_threads[i] = b.threads;
            out->bucket_max_n[i] = b.max_n;
            out->bucket_grid[i] = b.grid;
            out->bucket_dyn[i] = b.dyn;
        }
    }
    out->forked = p->buckets.size() > 1 ? p->forked : 0;
    return HP_OK;
}

hp_status hp_check(hp_plan_t plan) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p) return fail(HP_EINVAL, "null plan");
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    hipError_t e = hipDeviceSynchronize();
    int32_t flag = 0;
    if (e == hipSuccess) e = hipMemcpy(&flag, p->d_err, sizeof(flag), hipMemcpyDeviceToHost);
    // the flag stays raised from the failing run until it is reported here;
    // clearing it lets later runs wait for their data again
    if (e == hipSuccess && flag) e = launch_zero(reinterpret_cast<uint32_t *>(p->d_err), 1, nullptr);
    if (e == hipSuccess && flag) e = hipDeviceSynchronize();
    (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hp_check");
    if (flag) return fail(HP_EDEVICE, "a split workgroup timed out waiting for the others; results of the runs since the last check are void");
    return HP_OK;
}

hp_status hp_features(hp_plan_t plan, uint16_t *x, void *stream) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !x) return fail(HP_EINVAL, "null argument");
    if (p->K > 7 || p->total_vars < 1) return fail(HP_EINVAL, "bad plan");
    if (!p->d_feat_acc) {
        hipError_t e = hipMalloc((void **)&p->d_feat_acc, (size_t)p->total_vars * 20 * sizeof(float));
        if (e != hipSuccess) return hip_fail(e, "feature workspace");
    }
    hipError_t e = launch_features(*p, p->d_feat_acc, x, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "feature kernels");
    return HP_OK;
}

static bool mlp_ok(const hp_mlp *n) {
    return n && n->params && n->adam_m && n->adam_v && n->grad && n->w_bf16;
}

hp_status hp_mlp_sync(const hp_mlp *net, void *stream) {
    g_last_error.clear();
    if (!mlp_ok(net)) return fail(HP_EINVAL, "null network buffer");
    hipError_t e = launch_weights_to_bf16(*net, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "weight conversion");
    return HP_OK;
}

hp_status hp_mlp_forward(const hp_mlp *net, const uint16_t *x, int64_t rows, float *q, void *stream) {
    g_last_error.clear();
    if (!mlp_ok(net) || !x || !q) return fail(HP_EINVAL, "null argument");
    if (rows < 1) return fail(HP_EINVAL, "rows must be >= 1");
    hipError_t e = launch_mlp(*net, x, nullptr, rows, q, nullptr, false, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mlp forward");
    return HP_OK;
}

hp_status hp_mlp_backward(const hp_mlp *net, const uint16_t *x, const float *y, int64_t rows, float *loss_sum,
                          void *stream) {
    g_last_error.clear();
    if (!mlp_ok(net) || !net->partials || !x || !y || !loss_sum) return fail(HP_EINVAL, "null argument");
    if (rows < 1) return fail(HP_EINVAL, "rows must be >= 1");
    hipError_t e = launch_mlp(*net, x, y, rows, nullptr, loss_sum, true, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mlp backward");
    return HP_OK;
}

hp_status hp_mlp_adam(const hp_mlp *net, float lr, float beta1, float beta2, float eps, int64_t step, void *stream) {
    g_last_error.clear();
    if (!mlp_ok(net)) return fail(HP_EINVAL, "null network buffer");
    if (step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return fail(HP_EINVAL, "bad Adam hyperparameters");
    hipError_t e = launch_adam(*net, lr, beta1, beta2, eps, step, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "adam");
    return HP_OK;
}

hp_status hp_init_chains(hp_plan_t plan, const float *q, int32_t chain_lo, int32_t chain_hi, const hp_state *st,
                         void *stream) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !q || !st || !st->v) return fail(HP_EINVAL, "null argument");
    if (st->total_vars != p->total_vars || st->n_formulas != p->F || st->chains != p->B)
        return fail(HP_EINVAL, "state shape does not match the plan");
    if (chain_lo < 0 || chain_hi > p->B || chain_lo > chain_hi) return fail(HP_EINVAL, "bad chain range");
    hipError_t e = launch_init_chains(*p, q, chain_lo, chain_hi, st->v, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "init chains");
    return HP_OK;
}

hp_status hp_merge_candidates(hp_plan_t plan, const hp_state *st, const uint8_t *cand_v, void *stream) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !st || !cand_v || !st->v || !st->nu) return fail(HP_EINVAL, "null argument");
    if (st->total_vars != p->total_vars || st->n_formulas != p->F || st->chains != p->B ||
        st->nu_bytes != (p->precision == HP_FP32 ? 4 : 8))
        return fail(HP_EINVAL, "state shape does not match the plan");
    hipError_t e = launch_merge(*p, *st, cand_v, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "merge");
    return HP_OK;
}

hp_status hp_temper(hp_plan_t plan, const hp_state *st, int32_t parity, void *stream) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !st || !st->v || !st->t) return fail(HP_EINVAL, "null argument");
    if (st->total_vars != p->total_vars || st->n_formulas != p->F || st->chains != p->B)
        return fail(HP_EINVAL, "state shape does not match the plan");
    if (parity != 0 && parity != 1) return fail(HP_EINVAL, "parity must be 0 or 1");
    if (p->T > kMaxTemperTemps) return fail(HP_EUNSUPPORTED, "replica exchange handles up to 16 temperatures");
    hipError_t e = launch_temper(*p, *st, parity, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "replica exchange");
    return HP_OK;
}

hp_status hp_get_temps(hp_plan_t plan, int32_t *out, void *stream) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !out) return fail(HP_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(out, p->d_temp, (size_t)p->F * p->B * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "read temperatures");
    return HP_OK;
}

hp_status hp_chain_mean(hp_plan_t plan, const uint8_t *a, float *out, void *stream) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !a || !out) return fail(HP_EINVAL, "null argument");
    hipError_t e = launch_chain_mean(*p, a, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "chain mean");
    return HP_OK;
}

hp_status hp_philox_xor(uint64_t seed, int32_t formula, int64_t t, int32_t chain, int32_t phase, int64_t blocks,
                        int64_t n_out, uint32_t *out, void *stream) {
    g_last_error.clear();
    if (!out) return fail(HP_EINVAL, "null output");
    if (phase != 0 && phase != 1) return fail(HP_EINVAL, "phase must be 0 (hidden) or 1 (visible)");
    if (blocks < 1 || n_out < 1 || n_out > (int64_t(1) << 31) / blocks)
        return fail(HP_EINVAL, "need blocks >= 1, n_out >= 1 and n_out * blocks <= 2^31");
    hipError_t e = launch_philox_xor(seed, formula, t, chain, phase, blocks, n_out, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "philox kernel");
    return HP_OK;
}

hp_status hp_free(hp_plan_t plan) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p) return HP_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    hipError_t e = hipDeviceSynchronize();
    release(p);
    (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    return HP_OK;
}

}  // extern "C"
