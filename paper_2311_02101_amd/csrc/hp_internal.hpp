// Internal plan layout shared by the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hp.h"

namespace hp {

constexpr int kMaxK = 7;          // clause width limit (Sec. 3.1 assumes K <= 7)
constexpr int kMaxL = 8;          // hidden units per clause: K+1 <= 8
constexpr int kPatterns = 128;    // literal-truth patterns over K <= 7 inputs
constexpr int kHidMasks = 256;    // hidden-state masks over L <= 8 units
constexpr int kMaxVars = 32768;   // variable index packed in 15 bits
constexpr int kWave = 64;

// Per-formula descriptor (device copy).
struct FormulaDev {
    int32_t n;            // N_f
    int32_t c;            // C_f
    int64_t var_off;      // var_offset[f]: state block starts at var_off * B
    int64_t clause_off;   // clause_offset[f]: column of the packed clause table
    int64_t ptr_off;      // var_off + f: first of the N_f+1 occurrence offsets
};

struct WorkItem {
    int32_t f;            // formula
    int32_t b;            // chain within the formula
};

// Device tables prepared once per plan (per temperature tau):
//   thr[tau][m][l] = ceil(2^24 * sigma(b_c[l] + sum_k W_c[k,l] * bit_k(m)))
//       so that the hidden draw (word >> 8) < thr  <=>  U < p(h_l = 1 | m)
//       for the clause whose literal-truth pattern is m (eqs. 2, 4, 6);
//   G[tau][n][k]  = sum_{l ascending, bit_l(n)} W_c[k,l]
//       so that the contribution of clause c to its k-th input is
//       pol_kc * G[tau][h-mask][k]  (the vector l^(c) = W_f^(c) h^(c)).
struct DeviceTables {
    uint32_t *thr = nullptr;   // [T][128][8]
    double *g64 = nullptr;     // [T][256][8]
    float *g32 = nullptr;      // [T][256][8]
};

template <typename Real>
struct SweepParams {
    const FormulaDev *fd;
    const WorkItem *work;
    const uint16_t *lits;        // [K][ctot]: var index (15 bits) | negated << 15
    const uint32_t *csr_ptr;     // per formula N_f+1 absolute offsets into occ
    const uint32_t *occ;         // (c_local << 4) | (negated << 3) | k, (c, k) ascending
    const uint32_t *thr;         // [T][128][8]
    const Real *G;               // [T][256][8]
    const int32_t *temp_of_chain;
    uint8_t *v;
    Real *nu;
    int32_t *s_max;
    uint8_t *best;
    const int64_t *t_ptr;
    int64_t ctot;
    int64_t n_sweeps;
    Real alpha;
    uint32_t key0;
    uint32_t key1;               // xor-ed with the formula index
    int32_t K, L, B;
    int32_t lds_v_off;           // byte offsets inside dynamic LDS
    int32_t lds_hm_off;
};

struct Plan {
    int32_t F = 0, K = 0, L = 0, T = 0, B = 0;
    int32_t precision = HP_FP64;
    double alpha = 0.0;
    uint64_t seed = 0;
    int64_t total_vars = 0, total_clauses = 0, total_occ = 0;
    int32_t max_n = 0, max_c = 0;
    int32_t threads = 0;
    int32_t vpt = 0;             // visible groups of 4 per thread
    size_t lds_bytes = 0;
    int32_t lds_v_off = 0, lds_hm_off = 0;
    int device = 0;
    // device memory
    FormulaDev *d_fd = nullptr;
    WorkItem *d_work = nullptr;
    uint16_t *d_lits = nullptr;
    uint32_t *d_csr_ptr = nullptr;
    uint32_t *d_occ = nullptr;
    int32_t *d_temp = nullptr;
    double *d_W = nullptr;
    double *d_b = nullptr;
    DeviceTables tab;
    int32_t n_work = 0;
};

// kernels / launchers (hp_kernels.hip)
hipError_t launch_tables(const Plan &p, hipStream_t s);
hipError_t launch_sweep(const Plan &p, const hp_state &st, int64_t n_sweeps, hipStream_t s);

void set_error(const std::string &msg);

}  // namespace hp
