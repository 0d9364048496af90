// C-ABI entry points: validation, formula-RBM assembly (packing of the clause
// table and the per-variable occurrence lists), device allocation and launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
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
    (void)hipFree(p->d_fd);
    (void)hipFree(p->d_work);
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
    (void)hipFree(p->d_bar);
    (void)hipFree(p->d_err);
    (void)hipFree(p->d_temp);
    (void)hipFree(p->d_W);
    (void)hipFree(p->d_b);
    (void)hipFree(p->tab.thr);
    (void)hipFree(p->tab.g64);
    (void)hipFree(p->tab.g32);
    delete p;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

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
        case HP_EUNSUPPORTED: return "HP_EUNSUPPORTED: outside what this build handles";
    }
    return "unknown hp_status";
}

const char *hp_last_error(void) { return g_last_error.c_str(); }

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
    if (opts->precision == HP_MIXED_BF16)
        return fail(HP_EUNSUPPORTED, "mixed BF16 precision is not available in this build");
    if (opts->precision != HP_FP64 && opts->precision != HP_FP32)
        return fail(HP_EINVAL, "unknown precision");
    if (opts->threads != 0 && (opts->threads < kWave || opts->threads > 1024 || opts->threads % kWave))
        return fail(HP_EINVAL, "threads must be 0 or a multiple of 64 in [64, 1024]");
    if (opts->kernel < HP_KERNEL_AUTO || opts->kernel > HP_KERNEL_PUSH)
        return fail(HP_EINVAL, "unknown kernel variant");
    if (opts->split < 0 || opts->split > kMaxSplit || (opts->split & (opts->split - 1)))
        return fail(HP_EINVAL, "split must be 0 (automatic) or a power of two up to 16");
    for (int i = 0; i < T * K * L; ++i)
        if (!std::isfinite(rbm->W[i])) return fail(HP_EINVAL, "non-finite weight");
    for (int i = 0; i < T * L; ++i)
        if (!std::isfinite(rbm->b[i])) return fail(HP_EINVAL, "non-finite bias");
    std::vector<int32_t> temp(B);
    for (int b = 0; b < B; ++b) {
        temp[b] = opts->temp_of_chain ? opts->temp_of_chain[b] : (int32_t)((int64_t)b * T / B);
        if (temp[b] < 0 || temp[b] >= T) return fail(HP_EINVAL, "temperature index out of range");
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

    // --- clause table: padding normalisation + packing (idx | neg << 15) ---
    std::vector<uint16_t> lits((size_t)K * NC);
    std::vector<uint32_t> deg(NV, 0);
    for (int f = 0; f < F; ++f) {
        const int64_t n = cnf->var_offset[f + 1] - cnf->var_offset[f];
        for (int64_t c = cnf->clause_offset[f]; c < cnf->clause_offset[f + 1]; ++c) {
            int32_t first = 0;
            for (int k = 0; k < K; ++k)
                if (cnf->lits[(size_t)k * NC + c] != 0) {
                    first = cnf->lits[(size_t)k * NC + c];
                    break;
                }
            if (first == 0) return fail(HP_EINVAL, "clause " + std::to_string(c) + " has no literal");
            for (int k = 0; k < K; ++k) {
                int32_t x = cnf->lits[(size_t)k * NC + c];
                if (x == 0) x = first;
                const int64_t a = x < 0 ? -(int64_t)x : (int64_t)x;
                if (a > n) return fail(HP_EINVAL, "literal " + std::to_string(x) + " exceeds N_f");
                lits[(size_t)k * NC + c] = (uint16_t)((a - 1) | (x < 0 ? 0x8000u : 0u));
                deg[cnf->var_offset[f] + a - 1]++;
            }
        }
    }
    // --- per-variable occurrence lists, (c, k) ascending ---
    std::vector<uint32_t> csr_ptr(NV + F);
    std::vector<uint32_t> occ((size_t)K * NC);
    {
        uint64_t pos = 0;
        for (int f = 0; f < F; ++f) {
            const int64_t v0 = cnf->var_offset[f], n = cnf->var_offset[f + 1] - v0;
            for (int64_t i = 0; i < n; ++i) {
                csr_ptr[v0 + f + i] = (uint32_t)pos;
                pos += deg[v0 + i];
            }
            csr_ptr[v0 + f + n] = (uint32_t)pos;
        }
        std::vector<uint32_t> fill(NV + F);
        for (int64_t i = 0; i < NV + F; ++i) fill[i] = csr_ptr[i];
        for (int f = 0; f < F; ++f) {
            const int64_t v0 = cnf->var_offset[f], c0 = cnf->clause_offset[f];
            for (int64_t c = c0; c < cnf->clause_offset[f + 1]; ++c)
                for (int k = 0; k < K; ++k) {
                    const uint16_t e = lits[(size_t)k * NC + c];
                    const int64_t slot = v0 + f + (e & 0x7fff);
                    occ[fill[slot]++] = ((uint32_t)(c - c0) << 4) | ((e >> 15) << 3) | (uint32_t)k;
                }
        }
    }
    // --- push-kernel clause records: length, padding merge, sort by length ---
    // len = K minus the trailing run of copies of literal 0 (the padding of
    // Sec. 3.3); positions >= len contribute through the merged slot 0.
    std::vector<uint4> rec(NC);
    std::vector<uint32_t> orig(NC);
    std::vector<uint32_t> push_slots(NV, 0);
    std::vector<int32_t> negcnt(NV, 0);
    for (int f = 0; f < F; ++f) {
        const int64_t c0 = cnf->clause_offset[f], c1 = cnf->clause_offset[f + 1];
        std::vector<std::pair<int, int64_t>> key;
        key.reserve(c1 - c0);
        for (int64_t c = c0; c < c1; ++c) {
            int len = K;
            while (len > 1 && lits[(size_t)(len - 1) * NC + c] == lits[c]) --len;
            key.push_back({len, c});
            for (int k = 0; k < len; ++k) {
                const uint16_t e = lits[(size_t)k * NC + c];
                push_slots[cnf->var_offset[f] + (e & 0x7fff)]++;
                if (e >> 15) negcnt[cnf->var_offset[f] + (e & 0x7fff)]++;
            }
        }
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<int, int64_t> &a, const std::pair<int, int64_t> &b) {
                             return a.first < b.first;
                         });
        for (int64_t j = 0; j < c1 - c0; ++j) {
            const int len = key[j].first;
            const int64_t c = key[j].second;
            uint16_t sl[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            uint32_t negm = 0;
            for (int k = 0; k < K; ++k) sl[k] = lits[(size_t)k * NC + c];
            for (int k = 0; k < len; ++k) negm |= (uint32_t)(sl[k] >> 15) << k;
            sl[7] = (uint16_t)(len | (negm << 3));
            rec[c0 + j] = make_uint4(sl[0] | ((uint32_t)sl[1] << 16), sl[2] | ((uint32_t)sl[3] << 16),
                                     sl[4] | ((uint32_t)sl[5] << 16), sl[6] | ((uint32_t)sl[7] << 16));
            orig[c0 + j] = (uint32_t)(c - c0);
        }
    }
    // fixed-point scale: every slot contributes at most Wsum = sum |W_c| in
    // magnitude, a variable has at most max_slots slots, so |x| * 2^S stays
    // below 2^62 when (bound + 1) * 2^S < 2^62
    double wsum = 0.0;
    for (int t = 0; t < T; ++t) {
        double s = 0.0;
        for (int i = 0; i < K * L; ++i) s += std::fabs(rbm->W[(size_t)t * K * L + i]);
        wsum = std::max(wsum, s);
    }
    uint32_t max_slots = 1;
    for (int64_t i = 0; i < NV; ++i) max_slots = std::max(max_slots, push_slots[i]);
    const double bound = wsum * (double)max_slots * (1.0 + 1e-9) + 8.0;
    int fx_shift = 52;
    while (fx_shift > 0 && std::ldexp(bound + 1.0, fx_shift) >= std::ldexp(1.0, 62)) --fx_shift;

    // --- formula descriptors ---
    std::vector<FormulaDev> fd(F);
    for (int f = 0; f < F; ++f) {
        fd[f].n = (int32_t)(cnf->var_offset[f + 1] - cnf->var_offset[f]);
        fd[f].c = (int32_t)(cnf->clause_offset[f + 1] - cnf->clause_offset[f]);
        fd[f].var_off = cnf->var_offset[f];
        fd[f].clause_off = cnf->clause_offset[f];
        fd[f].ptr_off = cnf->var_offset[f] + f;
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
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { release(p); return hip_fail(e, "hipGetDevice"); }
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
    if (e != hipSuccess) { release(p); return hip_fail(e, "hipDeviceGetAttribute"); }
    const size_t real_bytes = opts->precision == HP_FP64 ? 8 : 4;
    const int threads = opts->threads ? opts->threads : kMaxThreads;
    p->threads = threads;

    // --- kernel variant per formula, work lists (largest formulas first) ---
    std::vector<int> order(F);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)fd[a].n * 7 + fd[a].c > (int64_t)fd[b].n * 7 + fd[b].c;
    });
    std::vector<WorkItem> work_push, work_pull;
    int pn = 0, qn = 0, qc = 0;   // largest N (push), largest N and C (pull)
    for (int f : order) {
        int32_t vo, xo, ho;
        const bool push_ok = fx_shift >= 40 && lds_bytes_push(fd[f].n, &vo, &xo) <= (size_t)max_lds;
        const bool pull_ok = lds_bytes_pull(fd[f].n, fd[f].c, real_bytes, &vo, &ho) <= (size_t)max_lds;
        bool use_push;
        if (opts->kernel == HP_KERNEL_PUSH) {
            if (!push_ok) {
                release(p);
                return fail(HP_EUNSUPPORTED, "push kernel: formula " + std::to_string(f) +
                                                 " does not fit in LDS (" + std::to_string(max_lds) + " B)");
            }
            use_push = true;
        } else if (opts->kernel == HP_KERNEL_PULL) {
            use_push = false;
        } else {
            use_push = push_ok;
        }
        if (!use_push && !pull_ok) {
            release(p);
            return fail(HP_EUNSUPPORTED, "formula " + std::to_string(f) +
                                             ": working set exceeds the workgroup LDS limit (" +
                                             std::to_string(max_lds) + " B)");
        }
        for (int b = 0; b < B; ++b) (use_push ? work_push : work_pull).push_back({f, b});
        if (use_push) pn = std::max(pn, fd[f].n);
        else { qn = std::max(qn, fd[f].n); qc = std::max(qc, fd[f].c); }
    }
    auto vpt_for = [&](int n) {
        const int groups = (n + 3) / 4;
        int v = 1;
        while (v * threads < groups) v *= 2;
        return v;
    };
    p->n_push = (int32_t)work_push.size();
    p->vpt_push = vpt_for(pn);
    p->vpt_pull = vpt_for(qn);
    p->lds_push = work_push.empty() ? 0 : lds_bytes_push(pn, &p->push_v_off, &p->push_x_off);
    p->lds_pull = work_pull.empty() ? 0 : lds_bytes_pull(qn, qc, real_bytes, &p->pull_v_off, &p->pull_hm_off);
    std::vector<WorkItem> work(work_push);
    work.insert(work.end(), work_pull.begin(), work_pull.end());
    p->n_work = (int32_t)work.size();

    // --- split: G co-resident workgroups per chain for the push items ---
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) { release(p); return hip_fail(e, "hipDeviceGetAttribute"); }
    int min_c = INT32_MAX;
    for (const WorkItem &it : work_push) min_c = std::min(min_c, fd[it.f].c);
    int G = 1;
    if (p->n_push > 0 && opts->split != 1) {
        const int occ = split_occupancy(*p);
        const int64_t capacity = (int64_t)cus * occ;
        if (opts->split >= 2) {
            G = opts->split;
            if ((int64_t)p->n_push * G > capacity) {
                release(p);
                return fail(HP_EUNSUPPORTED, "split " + std::to_string(G) + ": " +
                                                 std::to_string((int64_t)p->n_push * G) +
                                                 " workgroups cannot all be resident (capacity " +
                                                 std::to_string(capacity) + ")");
            }
        } else {
            // largest power of two that keeps every workgroup resident and
            // leaves each member at least 1024 clauses
            while (G * 2 <= kMaxSplit && (int64_t)p->n_push * G * 2 <= capacity &&
                   min_c / (G * 2) >= 1024)
                G *= 2;
        }
    }
    p->split = G;
    p->nstride = ((int64_t)pn + 15) / 16 * 16;
    p->xcd_map = (p->n_push % 8 == 0) ? 1 : 0;

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
    HP_TRY(upload(&p->d_lits, lits, s), "upload clause table");
    HP_TRY(upload(&p->d_csr_ptr, csr_ptr, s), "upload occurrence offsets");
    HP_TRY(upload(&p->d_occ, occ, s), "upload occurrences");
    HP_TRY(upload(&p->d_rec, rec, s), "upload clause records");
    HP_TRY(upload(&p->d_orig, orig, s), "upload clause order");
    HP_TRY(upload(&p->d_negcnt, negcnt, s), "upload negation counts");
    HP_TRY(upload(&p->d_temp, temp, s), "upload temperatures");
    HP_TRY(upload(&p->d_W, Wv, s), "upload W_c");
    HP_TRY(upload(&p->d_b, bv, s), "upload b_c");
    HP_TRY(hipMalloc((void **)&p->tab.thr, (size_t)T * kPatterns * kMaxL * sizeof(uint32_t)), "alloc thr");
    HP_TRY(hipMalloc((void **)&p->tab.g64, (size_t)T * kHidMasks * kMaxL * sizeof(double)), "alloc g64");
    HP_TRY(hipMalloc((void **)&p->tab.g32, (size_t)T * kHidMasks * kMaxL * sizeof(float)), "alloc g32");
    HP_TRY(hipMalloc((void **)&p->tab.gfx, (size_t)T * kHidMasks * kMaxL * sizeof(int64_t)), "alloc gfx");
    HP_TRY(hipMalloc((void **)&p->tab.gpad, (size_t)T * kMaxL * kHidMasks * sizeof(int64_t)), "alloc gpad");
    HP_TRY(hipMalloc((void **)&p->d_err, sizeof(int32_t)), "alloc error flag");
    HP_TRY(launch_zero(reinterpret_cast<uint32_t *>(p->d_err), 1, s), "clear error flag");
    HP_TRY(hipMalloc((void **)&p->d_tabflag, sizeof(int32_t)), "alloc table flag");
    HP_TRY(launch_zero(reinterpret_cast<uint32_t *>(p->d_tabflag), 1, s), "clear table flag");
    if (p->split > 1) {
        const size_t items = (size_t)p->n_push;
        HP_TRY(hipMalloc((void **)&p->d_xpart, items * p->split * p->nstride * sizeof(int64_t)), "alloc xpart");
        HP_TRY(hipMalloc((void **)&p->d_vbuf, items * p->nstride), "alloc vbuf");
        HP_TRY(hipMalloc((void **)&p->d_cnt, items * kMaxSplit * sizeof(int32_t)), "alloc counts");
        HP_TRY(hipMalloc((void **)&p->d_bar, items * 32 * sizeof(uint32_t)), "alloc barriers");
    }
    HP_TRY(launch_tables(*p, s), "table kernel");
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

hp_status hp_run(hp_plan_t plan, const hp_state *st, int64_t n_sweeps, void *stream) {
    g_last_error.clear();
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !st) return fail(HP_EINVAL, "null argument");
    if (n_sweeps < 0) return fail(HP_EINVAL, "n_sweeps must be >= 0");
    if (!st->v || !st->nu || !st->s_max || !st->best || !st->t) return fail(HP_EINVAL, "null state buffer");
    if (st->total_vars != p->total_vars || st->n_formulas != p->F || st->chains != p->B)
        return fail(HP_EINVAL, "state shape does not match the plan");
    const int want = p->precision == HP_FP64 ? 8 : 4;
    if (st->nu_bytes != want) return fail(HP_EINVAL, "nu element size does not match the precision");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != p->device) return fail(HP_EINVAL, "plan was built on another device");
    e = launch_sweep(*p, *st, n_sweeps, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
    return HP_OK;
}

hp_status hp_plan_query(hp_plan_t plan, hp_plan_info *out) {
    g_last_error.clear();
    const Plan *p = reinterpret_cast<const Plan *>(plan);
    if (!p || !out) return fail(HP_EINVAL, "null argument");
    out->threads = p->threads;
    out->split = p->split;
    out->push_items = p->n_push;
    out->pull_items = p->n_work - p->n_push;
    out->fx_shift = p->fx_shift;
    out->reserved = 0;
    out->lds_push = (int64_t)p->lds_push;
    out->lds_pull = (int64_t)p->lds_pull;
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
    (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hp_check");
    if (flag) return fail(HP_EDEVICE, "a cross-workgroup barrier timed out; results of the affected runs are void");
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
