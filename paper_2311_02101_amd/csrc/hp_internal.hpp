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
constexpr int kThrRows = 2 * kPatterns;   // push kernels: rows 2^len + (pattern of the len literals)
constexpr int kRowWords = 16;     // contribution table row: 8 slot words, 8 merged-padding words
constexpr int kHidMasks = 256;    // hidden-state masks over L <= 8 units
constexpr int kMaxVars = 32768;   // variable index packed in 15 bits
constexpr int kWave = 64;
constexpr int kMaxThreads = 1024;

// Per-formula descriptor (device copy).
struct FormulaDev {
    int32_t n;            // N_f
    int32_t c;            // C_f
    int64_t var_off;      // var_offset[f]: state block starts at var_off * B
    int64_t clause_off;   // clause_offset[f]: first clause record / column
    int64_t ptr_off;      // var_off + f: first of the N_f+1 occurrence offsets
    int32_t lofs[8];      // push records (sorted by length) of length <= k, k = 0..7
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
//       pol_kc * G[tau][h-mask][k]  (the vector l^(c) = W_f^(c) h^(c));
//   gfx[tau][n][k] = round(G * 2^S) as int64 (fixed point, scale 2^S) for
//       k < 8, and gfx[tau][n][8 + len] = gfx[n][0] + sum_{k = len}^{K-1}
//       gfx[n][k] for len = 1..K: the merged contribution of a clause's
//       first literal and its padding copies (Sec. 3.3 pads by repeating a
//       literal); rows n >= 2^L repeat row n mod 2^L.
struct DeviceTables {
    uint32_t *thr = nullptr;   // [T][128][8]
    double *g64 = nullptr;     // [T][256][8]
    float *g32 = nullptr;      // [T][256][8]
    int64_t *gfx = nullptr;    // [T][256][16] (size-clustered model: its own layout)
    int64_t *gpad = nullptr;   // size-clustered model only
    uint4 *mfma = nullptr;     // [T][2][64] per-lane BF16 limb operands (mixed precision)
};

// Mixed-precision contraction operands.  Both per-clause products are MFMA
// v_mfma_f32_32x32x16_bf16 with the clauses as the 32 columns and the
// constant weights as the 32 x 16 A operand:
//   hidden logits   z[u]  = b[u] + sum_k lit[k] W[k][u]  (bias as input 7 = 1)
//                   A rows (g, u) = 8g + u, K index = (h, k) = 8h + k
//   contributions   l[k]  = sum_u h[u] W[k][u]
//                   A rows (g, k) = 8g + k, K index = (h, u) = 8h + u
// Entry (g, h) holds BF16 limb j = 2g + h of the weight.  Limbs of one
// column share the exponent grid of the column's largest magnitude 2^E:
// limb j is a multiple of 2^(E - 8(j+1)) of magnitude <= 2^(E - 8j), so a
// product over 8 binary inputs of one limb pair (g) is exact in FP32 and the
// four pairs carry 64 bits of every weight.
constexpr int kLimbs = 8;

// Size-clustered model (Sec. 4): one canonical RBM per clause size K = 3..7
// with L = 3 hidden units for K = 3 and K + 1 otherwise; a clause of length
// len uses the RBM of K = max(len, 3), its inputs padded to K by repeating
// literal 0.  Per temperature the tables of the five groups are concatenated
// with closed-form offsets:
//   thr   rows [248][8]  group K at row 2^K - 8           (2^K patterns)
//   gfx   rows [488][8]  group K at row 0 (K = 3), else 2^(K+1) - 24
//                                                      (2^L hidden masks)
//   gpad  [504]          length len at 8 (len - 1) (len <= 3), else
//                        2^(len+1) - 8                   (2^L masks each)
// gpad holds the merged contribution of literal 0 and its padding copies
// (slots len..K-1) of a clause of that length.
constexpr int kClustGroups = 5;
constexpr int kClustThrRows = 248;
constexpr int kClustGfxRows = 488;
constexpr int kClustGpad = 504;
__host__ __device__ constexpr int clust_hidden(int K) { return K == 3 ? 3 : K + 1; }

// clause length and negation bits from a record's last word (layout below)
__device__ __forceinline__ uint32_t rec_len(uint32_t w) {
    return (w >> 16) != 0u ? 7u : 31u - (uint32_t)__clz((int)w);
}
__device__ __forceinline__ uint32_t rec_negm(uint32_t w) {
    return (w >> 16) != 0u ? (w >> 19) : (w ^ (1u << rec_len(w)));
}

// device pointers of the size RBMs (nullptr for a group no clause uses)
struct ClustRbm {
    const double *W[kClustGroups];   // [T][K][L] of K = 3 + i
    const double *b[kClustGroups];   // [T][L]
};

// Clause record of the push kernel: 8 x 16-bit slots in a uint4.  Slots
// 0..len-1 hold literal k as (0-based variable index) | (negated << 15),
// where len is the clause length (positions >= len repeat literal 0).  The
// last word holds, for len = 7, slot 6 and then len | (negation bits) << 3
// in the high half; below seven literals it is the negation bits | 2^len
// alone, so its XOR with the literals' values is the push kernels'
// threshold row 2^len + pattern.  Records of a formula
// are sorted by len (stable); orig[] keeps the first Philox block of the
// clause's hidden draw, its index in the input times the blocks per clause,
// which addresses its random numbers.
//
// thr[tau][m][l] holds 256 * ceil(2^24 p) - 1 (see the table kernel).

template <typename Real>
struct SweepParams {
    const FormulaDev *fd;
    const WorkItem *work;
    const uint16_t *lits;        // pull: [K][ctot] var index (15 bits) | negated << 15
    const uint32_t *csr_ptr;     // pull: per formula N_f+1 absolute offsets into occ
    const uint32_t *occ;         // pull: (c_local << 4) | (negated << 3) | k, (c, k) ascending
    const uint4 *rec;            // push: clause records [ctot]
    const uint32_t *orig;        // push: first Philox block of the record's hidden draw [ctot]
    const int32_t *negcnt;       // push: negated slots per variable [sum N]
    const uint32_t *thr;         // [T][128][8]
    const Real *G;               // [T][256][8]
    const int64_t *gfx;          // [T][256][16] contribution rows (size-clustered: its layout)
    const int64_t *gpad;         // size-clustered model's merged paddings
    const uint4 *mfma;           // [T][2][64] mixed-precision A operands
    const int32_t *temp_of_chain;  // [F][B] temperature index per (formula, chain)
    uint8_t *v;
    Real *nu;
    int32_t *s_max;
    uint8_t *best;
    const int64_t *t_ptr;
    int64_t ctot;
    int64_t n_sweeps;
    Real alpha;
    double fx_scale;             // 2^-S
    uint32_t key0;
    uint32_t key1;               // xor-ed with the formula index
    int32_t K, L, B;
    int32_t lds_v_off;           // byte offsets inside dynamic LDS
    int32_t lds_hm_off;          // pull: hidden masks
    int32_t lds_x_off;           // push: int64 accumulators
    int32_t dyn_steps;           // clause phase: 1 = steps from a workgroup counter, 0 = round-robin
};

// Split launch: the G workgroups of one chain exchange, every sweep, their
// partial fixed-point logits (xpart) and the owners' new values (vbuf).
constexpr int kMaxSplit = 16;

struct SplitParams {
    int64_t *xpart;              // [items][G][nstride]
    uint8_t *vbuf;               // [items][nstride]
    int32_t *cnt;                // [items][2][kMaxSplit] partial clause counts by sweep parity
    int32_t *err;                // [1] exchange time-out flag
    int64_t nstride;
    int32_t G;
    uint32_t wait_limit;         // reloads of a mailbox word before giving up
    int32_t xcd_map;             // members of an item on the same XCD
    int32_t n_xcd;
};

enum class Variant { kPull = 0, kPush = 1 };

// A launch over a contiguous range of work items: formulas of one size class
// and one kernel variant, with its own workgroup size and LDS footprint.
// push: every table in LDS; mid: the merged padding words read from global
// memory (one read per clause), the rest in LDS; wide: the contribution
// rows in global memory (the largest formulas)
// XCDs of the GPU (MI355X: 8 compute dies, each with its own L2); workgroup
// w of a launch is dispatched to XCD w mod 8
constexpr int kXcds = 8;
// work counters of one launch: one per XCD, each on its own 128-byte line
constexpr int kQueueWords = kXcds * 32;

// Work queue of a persistent launch: ctr == nullptr runs item w on
// workgroup w; else workgroups take items of their own XCD's range first,
// then help the other XCDs' ranges.
struct WorkQueue {
    uint32_t *ctr;               // [kXcds][32] counters, zeroed before the launch
    int32_t count;               // items of the launch
    int32_t xq[kXcds + 1];       // item ranges per XCD
};

enum BucketKind : int32_t { kBucketPush = 0, kBucketWide = 1, kBucketPull = 2, kBucketMid = 3 };
constexpr int kMaxBuckets = 32;

struct Bucket {
    int32_t kind = kBucketPush;
    int32_t first = 0, count = 0;   // work items [first, first + count)
    int32_t threads = 0, vpt = 1;   // workgroup size, visible groups per thread
    int32_t max_n = 0, max_c = 0;
    size_t lds = 0;
    int32_t v_off = 0, x_off = 0, hm_off = 0;
    int32_t grid = 0;               // persistent grid (0: one workgroup per item)
    int32_t dyn = 1;                // clause-phase steps from a counter (1) or round-robin (0)
    // persistent grids: the items are grouped by XCD, [xq[x], xq[x+1]) for
    // XCD x (offsets from `first`); whole formulas per XCD, balanced by work
    int32_t xq[kXcds + 1] = {};
};

struct GraphEntry {
    void *v, *nu, *s_max, *best, *t;
    int64_t n_sweeps;
    hipGraphExec_t exec;
};

struct Plan {
    int32_t F = 0, K = 0, L = 0, T = 0, B = 0;
    int32_t precision = HP_FP64;
    double alpha = 0.0;
    uint64_t seed = 0;
    int64_t total_vars = 0, total_clauses = 0, total_occ = 0;
    int32_t max_n = 0, max_c = 0;
    int32_t threads = 0;         // workgroup size override (0 = per bucket)
    int32_t fx_shift = 0;        // S of the fixed-point accumulators
    int32_t cus = 0;             // compute units of the device
    std::vector<Bucket> buckets;
    int32_t split = 1;           // G workgroups per chain (single push bucket only)
    int32_t wait_limit = 0;      // split: mailbox reloads before giving up (0 = default)
    int32_t xcd_map = 0;
    int64_t nstride = 0;
    int32_t use_graph = 0;
    int32_t forked = 1;          // several buckets: forked over side streams (1) or in sequence (0)
    int32_t clust = 0;           // size-clustered model: tables in the clustered layout
    ClustRbm crbm = {};          // its RBMs (device copies in d_Wc / d_bc)
    double *d_Wc = nullptr;
    double *d_bc = nullptr;
    int device = 0;
    hipStream_t side[kMaxBuckets] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[kMaxBuckets] = {};
    hipStream_t cap_stream = nullptr;
    std::vector<GraphEntry> graphs;
    uint32_t *d_queue = nullptr;     // [kMaxBuckets][kQueueWords] persistent work counters
    int64_t *d_var_off = nullptr;    // [F+1]
    int64_t *d_clause_off = nullptr; // [F+1]
    float *d_feat_acc = nullptr;     // feature workspace, allocated on first use
    // device memory
    FormulaDev *d_fd = nullptr;
    WorkItem *d_work = nullptr;
    WorkItem *d_work_fb = nullptr;        // the same items in (formula, chain) order
    int32_t *d_mg_cnt = nullptr;          // merge: counts (current, returned), source rows
    uint8_t *d_mg_v = nullptr;            // merge: staging of v and nu (allocated on first use)
    unsigned char *d_mg_nu = nullptr;
    uint16_t *d_lits = nullptr;
    uint32_t *d_csr_ptr = nullptr;
    uint32_t *d_occ = nullptr;
    uint4 *d_rec = nullptr;
    uint32_t *d_orig = nullptr;
    int32_t *d_negcnt = nullptr;
    int32_t *d_tabflag = nullptr;
    int32_t *d_temp = nullptr;            // [F][B]
    double *d_fe = nullptr;               // replica exchange: [T][128] clause free energies,
    double *d_fe_chain = nullptr;         //   [F][B][T] formula free energies,
    int32_t *d_temp_old = nullptr;        //   [F][B] temperatures before the round
    double *d_W = nullptr;
    double *d_b = nullptr;
    DeviceTables tab;
    int32_t n_work = 0;
    int64_t *d_xpart = nullptr;
    uint8_t *d_vbuf = nullptr;
    int32_t *d_cnt = nullptr;
    int32_t *d_err = nullptr;
};

// Device buffers of one run beyond its inputs and outputs: the persistent
// launches' work counters and the split launch's exchange mailboxes.  hp_run
// uses the plan's own; hp_run_noalloc carves them out of the library's static
// scratch array (kScratchBytes per device).
struct RunBuffers {
    uint32_t *queue;             // [kMaxBuckets][kQueueWords] work counters
    int64_t *xpart;              // split: [items][G][nstride] partial logits
    uint8_t *vbuf;               // split: [items][nstride] packed new values
    int32_t *cnt;                // split: [items][2][kMaxSplit] partial counts
};
constexpr size_t kScratchBytes = size_t(16) << 20;
RunBuffers plan_buffers(const Plan &p);
// bytes of static scratch a run of this plan needs, and its layout there
size_t run_scratch_bytes(const Plan &p);
RunBuffers scratch_buffers(const Plan &p, void *base);
// Resolve this device's address of the static scratch array (once per
// device, with the device current); static_scratch returns it afterwards
// (nullptr if it was never resolved on that device).
hipError_t static_scratch_init(int device);
void *static_scratch(int device);

// kernels / launchers (hp_kernels.hip)
hipError_t launch_tables(const Plan &p, hipStream_t s);
hipError_t launch_sweep(const Plan &p, const hp_state &st, int64_t n_sweeps, hipStream_t s);
hipError_t launch_sweep(const Plan &p, const hp_state &st, int64_t n_sweeps, hipStream_t s, const RunBuffers &rb);
// the launches of a run without the sweep-counter advance
hipError_t launch_buckets(const Plan &p, const hp_state &st, int64_t n_sweeps, hipStream_t s, const RunBuffers &rb);
// one bucket alone (no fork/join, no counter advance): used by the tuner
hipError_t launch_bucket(const Plan &p, const Bucket &b, const hp_state &st, int64_t n_sweeps, hipStream_t s);
// raise the dynamic-LDS limit of every sweep kernel to `bytes` (once per plan)
hipError_t set_kernel_lds_limits(int bytes);
// resident workgroups per CU of a bucket's kernel at its launch shape
int bucket_occupancy(const Plan &p, const Bucket &b);

hipError_t launch_zero(uint32_t *p, int64_t n, hipStream_t s);
hipError_t launch_philox_xor(uint64_t seed, int32_t formula, int64_t t, int32_t chain, int32_t phase, int64_t blocks,
                             int64_t n_out, uint32_t *out, hipStream_t s);

// owned variables per thread of a split member (1 or 2 in registers, else
// 0) for the largest formula, G members and the given workgroup size
int split_vpt(int max_n, int G, int threads);
// resident workgroups per CU of the split kernel variant that a launch with G
// members per chain runs (the VPT of split_vpt) at this plan's shape
int split_occupancy(const Plan &p, int G);

// LDS bytes of the two kernel variants for the largest formula
size_t lds_bytes_pull(int max_n, int max_c, size_t real_bytes, int32_t *v_off, int32_t *hm_off);
size_t lds_bytes_push(int max_n, int kind, int32_t *v_off, int32_t *x_off);
size_t lds_bytes_clust(int max_n, int32_t *v_off, int32_t *x_off);

// learned initial assignments (hp_mlp.hip)
hipError_t launch_features(const Plan &p, float *acc, uint16_t *x, hipStream_t s);
hipError_t launch_mlp(const hp_mlp &net, const uint16_t *x, const float *y, int64_t rows, float *q,
                      float *loss_sum, bool backward, hipStream_t s);
hipError_t launch_adam(const hp_mlp &net, float lr, float beta1, float beta2, float eps, int64_t step,
                       hipStream_t s);
hipError_t launch_weights_to_bf16(const hp_mlp &net, hipStream_t s);
hipError_t launch_init_chains(const Plan &p, const float *q, int chain_lo, int chain_hi, uint8_t *v,
                              hipStream_t s);
hipError_t launch_chain_mean(const Plan &p, const uint8_t *a, float *out, hipStream_t s);
hipError_t launch_merge(Plan &p, const hp_state &st, const uint8_t *cand, hipStream_t s);
constexpr int kMaxTemperTemps = 16;
hipError_t launch_temper(Plan &p, const hp_state &st, int parity, hipStream_t s);

void set_error(const std::string &msg);

}  // namespace hp
