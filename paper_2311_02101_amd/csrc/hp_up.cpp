// Prioritized unit propagation on the host (Sec. 3.4).
//
// The sampled assignments of a formula's chains are improved on CPU threads
// while the GPU keeps sampling.  For one chain:
//   1. variables ordered by the variance average nu, highest first, ties by
//      index;
//   2. the first floor(N/2) of that order keep their sampled values;
//   3. every clause is examined once in clause order: a clause with no true
//      literal and exactly one unassigned literal makes that literal true
//      (its variable is assigned and queued); one with no true and no
//      unassigned literal is a conflict and stays unsatisfied;
//   4. FIFO propagation: for a variable taken from the queue, every clause in
//      which its literal is false is examined as in 3, in clause order;
//   5. the remaining variables in priority order: one still unassigned takes
//      its sampled value, is queued and propagated as in 4.
// A clause is the set of its distinct literals.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "hp.h"

namespace hp {
void set_error(const std::string &msg);
}

namespace {

struct UpFormula {
    int32_t n = 0;
    std::vector<int32_t> cl_ptr;   // [C+1] into lit
    std::vector<int32_t> lit;      // distinct literals, signed 1-based
    std::vector<int32_t> occ_ptr;  // [N+1] into occ
    std::vector<int32_t> occ;      // per variable, in clause order, once per
                                   // distinct literal: clause << 1 | negated
};

// Builds the clause and occurrence lists of formula f; false on a bad table.
bool build_formula(const hp_cnf *cnf, int f, UpFormula &F, std::string &err) {
    const int K = cnf->k;
    const int64_t NC = cnf->clause_offset[cnf->n_formulas];
    const int64_t c0 = cnf->clause_offset[f], c1 = cnf->clause_offset[f + 1];
    const int64_t n = cnf->var_offset[f + 1] - cnf->var_offset[f];
    if (n < 1 || c1 < c0) {
        err = "empty formula";
        return false;
    }
    F.n = (int32_t)n;
    F.cl_ptr.assign(1, 0);
    F.lit.clear();
    std::vector<int32_t> cnt(n + 1, 0);
    for (int64_t c = c0; c < c1; ++c) {
        int32_t first = 0;
        for (int k = 0; k < K && !first; ++k) first = cnf->lits[(size_t)k * NC + c];
        if (!first) {
            err = "clause " + std::to_string(c - c0) + " of formula " + std::to_string(f) + " has no literal";
            return false;
        }
        const size_t start = F.lit.size();
        for (int k = 0; k < K; ++k) {
            int32_t l = cnf->lits[(size_t)k * NC + c];
            if (l == 0) l = first;                       // padding: the first literal
            if (l < -n || l > n) {
                err = "literal exceeds the formula's variable count";
                return false;
            }
            bool seen = false;
            for (size_t j = start; j < F.lit.size(); ++j) seen |= F.lit[j] == l;
            if (!seen) {
                F.lit.push_back(l);
                cnt[std::abs(l) - 1 + 1]++;
            }
        }
        F.cl_ptr.push_back((int32_t)F.lit.size());
    }
    F.occ_ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) F.occ_ptr[i + 1] = F.occ_ptr[i] + cnt[i + 1];
    F.occ.assign(F.occ_ptr[n], 0);
    std::vector<int32_t> fill(F.occ_ptr.begin(), F.occ_ptr.end() - 1);
    const int32_t C = (int32_t)(F.cl_ptr.size() - 1);
    for (int32_t c = 0; c < C; ++c)
        for (int32_t j = F.cl_ptr[c]; j < F.cl_ptr[c + 1]; ++j)
            F.occ[fill[std::abs(F.lit[j]) - 1]++] = (c << 1) | (F.lit[j] < 0 ? 1 : 0);
    return true;
}

struct UpWork {
    std::vector<int32_t> order;
    std::vector<int8_t> val;       // -1 unassigned, else 0 / 1
    std::vector<int32_t> queue;
};

inline int lit_value(const std::vector<int8_t> &val, int32_t l) {
    const int8_t x = val[std::abs(l) - 1];
    if (x < 0) return -1;
    return l > 0 ? x : 1 - x;
}

void up_chain(const UpFormula &F, const uint8_t *v, const double *nu, uint8_t *out, UpWork &w) {
    const int32_t n = F.n;
    const int32_t C = (int32_t)(F.cl_ptr.size() - 1);
    w.order.resize(n);
    std::iota(w.order.begin(), w.order.end(), 0);
    std::sort(w.order.begin(), w.order.end(), [nu](int32_t a, int32_t b) {
        return nu[a] > nu[b] || (nu[a] == nu[b] && a < b);
    });
    w.val.assign(n, -1);
    w.queue.clear();
    size_t head = 0;
    auto examine = [&](int32_t c) {
        int32_t free_lit = 0, n_free = 0;
        for (int32_t j = F.cl_ptr[c]; j < F.cl_ptr[c + 1]; ++j) {
            const int x = lit_value(w.val, F.lit[j]);
            if (x == 1) return;
            if (x < 0) {
                ++n_free;
                free_lit = F.lit[j];
            }
        }
        if (n_free == 1) {
            const int32_t i = std::abs(free_lit) - 1;
            w.val[i] = free_lit > 0 ? 1 : 0;
            w.queue.push_back(i);
        }
    };
    auto propagate = [&]() {
        while (head < w.queue.size()) {
            const int32_t i = w.queue[head++];
            // clauses in which the literal of i is false: the positive ones
            // when i = 0, the negated ones when i = 1 (a clause holding both
            // literals is examined once, from the false one, and is satisfied)
            const int32_t false_neg = w.val[i];
            for (int32_t j = F.occ_ptr[i]; j < F.occ_ptr[i + 1]; ++j)
                if ((F.occ[j] & 1) == false_neg) examine(F.occ[j] >> 1);
        }
    };
    const int32_t half = n / 2;
    for (int32_t r = 0; r < half; ++r) w.val[w.order[r]] = (int8_t)(v[w.order[r]] & 1);
    for (int32_t c = 0; c < C; ++c) examine(c);
    propagate();
    for (int32_t r = half; r < n; ++r) {
        const int32_t i = w.order[r];
        if (w.val[i] < 0) {
            w.val[i] = (int8_t)(v[i] & 1);
            w.queue.push_back(i);
            propagate();
        }
    }
    for (int32_t i = 0; i < n; ++i) out[i] = (uint8_t)w.val[i];
}

}  // namespace

extern "C" {

hp_status hp_unit_propagate(const hp_cnf *cnf, int32_t formula, int32_t n_chains, const uint8_t *v,
                            const double *nu, uint8_t *out, int32_t threads) {
    hp::set_error("");
    if (!cnf || !v || !nu || !out || !cnf->var_offset || !cnf->clause_offset || !cnf->lits) {
        hp::set_error("null argument");
        return HP_EINVAL;
    }
    if (cnf->k < 1 || cnf->k > 7 || formula < 0 || formula >= cnf->n_formulas || n_chains < 0 || threads < 0) {
        hp::set_error("bad formula index, K, chain or thread count");
        return HP_EINVAL;
    }
    UpFormula F;
    std::string err;
    if (!build_formula(cnf, formula, F, err)) {
        hp::set_error(err);
        return HP_EINVAL;
    }
    const int64_t n = F.n;
    int T = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
    T = std::max(1, std::min(T, n_chains));
    auto work = [&](int t) {
        UpWork w;
        for (int b = t; b < n_chains; b += T) up_chain(F, v + (size_t)b * n, nu + (size_t)b * n, out + (size_t)b * n, w);
    };
    if (T == 1) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        pool.reserve(T);
        for (int t = 0; t < T; ++t) pool.emplace_back(work, t);
        for (std::thread &th : pool) th.join();
    }
    return HP_OK;
}

}  // extern "C"
