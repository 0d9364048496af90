/*
 * hp.h -- C ABI of the RbmSAT block-Gibbs hot path on MI355X (gfx950).
 *
 * The method (Sec. 3 of "Solving MaxSAT with Matrix Multiplication"): a CNF
 * formula becomes a product of clause-RBMs (Sec. 3.1), one canonical OR-gate
 * RBM (W_c, b_c) per temperature mapped onto every clause by the negation
 * transform (eq. 4); B parallel Markov chains then run block Gibbs sampling
 * (eqs. 2-3, factorised as eqs. 6-7) and keep the best assignment seen
 * (Sec. 3.2).  One sweep, per chain: gather the clause inputs, count the
 * satisfied clauses, track the best, sample the hidden units of every clause,
 * scatter-add the per-clause logit contributions onto the variables, update
 * the conditional-variance moving average (Sec. 3.4) and sample new values.
 *
 * Conventions
 *   - Every function returns an hp_status (0 = success, < 0 = error); no C++
 *     exception crosses this boundary.  hp_last_error() returns a message for
 *     the last failure on the calling thread.
 *   - "host" pointers are read during the call only and may be freed when it
 *     returns; "device" pointers are HIP device memory owned by the caller.
 *   - Streams are hipStream_t passed as void*; NULL is the null stream.  All
 *     device work is enqueued on that stream; nothing synchronises the host.
 *   - A batch may hold several formulas of different sizes.  Formula f has
 *     N_f = var_offset[f+1]-var_offset[f] variables and
 *     C_f = clause_offset[f+1]-clause_offset[f] clauses, and B chains.  Its
 *     per-chain arrays occupy the [B][N_f] row-major block starting at element
 *     var_offset[f]*B of the batch-wide arrays.
 */
#ifndef HP_H
#define HP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HP_OK = 0,
    HP_EINVAL = -1,        /* invalid argument; nothing was allocated or enqueued */
    HP_ENOMEM = -2,        /* device allocation failed                            */
    HP_EDEVICE = -3,       /* a HIP runtime call failed                           */
    HP_EUNSUPPORTED = -4   /* valid input outside what the library handles       */
} hp_status;

/* Arithmetic of the sweep.  HP_FP64 and HP_FP32 take the hidden draws from
 * per-temperature threshold tables and the contributions from fixed-point
 * tables (both prepared in FP64); the visible sigmoid and variance EMA run in
 * the named precision.  HP_MIXED_BF16 is the form of the appendix
 * ("Precision"), where the accelerator multiplies in bfloat16: per clause, the
 * hidden logits z = b + W^T lit and the contributions l = W h are computed
 * every sweep as v_mfma_f32_32x32x16_bf16 products with W split into eight
 * BF16 limbs (each limb pair exact in FP32, four pairs = 64 bits), hidden
 * draws decided from an FP32 sigmoid unless U is within 16 * 2^-24 of it
 * (then the FP64 threshold decides), contributions recombined in FP64 onto
 * the fixed-point grid; visible update and EMA in FP64, nu is double.  Its
 * samples equal HP_FP64's.  It runs the push launch only (no pull kernel, no
 * split) and returns HP_EUNSUPPORTED otherwise. */
typedef enum {
    HP_FP64 = 0,
    HP_FP32 = 1,
    HP_MIXED_BF16 = 2
} hp_precision;

/* The formula batch: signed 1-based literal table (Sec. 3.3).  Column c of
 * lits lists the literals of clause c; the sign is the polarity, so the
 * column (1, 2, -3, 4) is v1 or v2 or (not v3) or v4.  A 0 entry is padding
 * (Sec. 3.1) and is replaced by the clause's first non-zero literal, i.e.
 * the clause is padded by repeating a literal with the same polarity
 * (Sec. 3.3), which keeps its satisfying set. */
typedef struct {
    int32_t n_formulas;             /* F >= 1                                          */
    const int64_t *var_offset;      /* host [F+1], prefix sums of N_f, var_offset[0]=0 */
    const int64_t *clause_offset;   /* host [F+1], prefix sums of C_f                  */
    int32_t k;                      /* padded clause width K, 1..7                     */
    const int32_t *lits;            /* host [K][sum C_f], clause-minor; literals of
                                       formula f are 1-based within that formula      */
} hp_cnf;

/* Canonical OR-gate RBMs, one per temperature (Sec. 3.1 "OR gate as an
 * RBM", the free-energy target F* acts as the temperature; appendix
 * "Pretraining": L = 3 for K = 3, L = K+1 for K in [4,7]).  The visible bias
 * is zero (Sec. 3.1). */
typedef struct {
    int32_t k, l, n_temps;          /* K (must equal hp_cnf.k), L in 1..8, n_temps >= 1 */
    const double *W;                /* host [n_temps][K][L]  canonical weights W_c     */
    const double *b;                /* host [n_temps][L]     canonical hidden bias b_c */
} hp_rbm;

typedef struct {
    int32_t chains;                 /* B chains per formula (the "batch size"), >= 1   */
    const int32_t *temp_of_chain;   /* host [B] initial temperature index of chain b of
                                       every formula, or NULL: floor(b*n_temps/B);
                                       hp_temper changes them per formula             */
    int32_t precision;              /* hp_precision                                    */
    double alpha;                   /* variance moving-average rate, in [0, 1]         */
    uint64_t seed;                  /* Philox key source                               */
    int32_t threads;                /* workgroup size override (0 = automatic)         */
    int32_t split;                  /* workgroups per chain of the push kernel: 0 =
                                       automatic (fill the device), 1 = one, or a power
                                       of two up to 16.  The plan admits a split only
                                       if all its workgroups fit on the device at once
                                       and every formula has more than 4 (split - 1)
                                       variables (HP_EUNSUPPORTED otherwise); they
                                       exchange data every sweep, so a split run must
                                       not share the device with work that keeps CUs
                                       occupied for long (its bounded waits for the
                                       other workgroups would time out: hp_check)    */
    int32_t kernel;                 /* hp_kernel: sweep kernel variant                 */
    int32_t graph;                  /* 1: hp_run replays a captured hipGraph of its
                                       launches (cached per state buffers and sweep
                                       count); incompatible with split > 1           */
    const hp_rbm *size_rbms;        /* NULL: every clause uses `rbm` (padded to K).
                                       Else the size-clustered model (Sec. 4): host
                                       [5] canonical RBMs for K = 3..7 (k = 3+i,
                                       l = 3 for K = 3 else K+1, n_temps as `rbm`);
                                       a clause of length l (its column without the
                                       trailing copies of its first literal) uses
                                       the K = max(l, 3) RBM, lengths 1..2 padded by
                                       the first literal; hidden unit j of clause c
                                       draws block 2c + j/4.  Push launches only (no
                                       pull kernel, no mixed precision).            */
    int32_t split_wait_limit;       /* split launches: 0 = wait about a second for
                                       another workgroup's data before giving up;
                                       > 0 = reloads of a word before giving up (a
                                       tiny limit forces the failure path that
                                       hp_check reports, for tests)                  */
} hp_opts;

typedef enum {
    HP_KERNEL_AUTO = 0,             /* fixed-point push when it fits in LDS, else pull */
    HP_KERNEL_PULL = 1,             /* per-variable occurrence lists, FP sums in the
                                       order (clause, position) ascending             */
    HP_KERNEL_PUSH = 2              /* clause-side scatter into int64 fixed-point LDS
                                       accumulators (exact, order-independent sums)   */
} hp_kernel;

/* Chain state: caller-owned DEVICE buffers in the layout described above.
 * The randomness of sweep t comes from Philox4x32-10 (Salmon et al., SC'11)
 * with key (seed mod 2^32, (seed div 2^32) xor f) and counter
 * (t mod 2^32, chain, phase*2^31 + block, t div 2^32): hidden unit l of
 * clause c uses block c*ceil(L/4) + l/4 of phase 0, visible unit i uses block
 * i/4 of phase 1, and word j%4 of the block becomes U = (word >> 8) * 2^-24;
 * a unit is set iff U < its conditional probability.  Because draws are
 * addressed by the absolute sweep t, hp_run(S1) followed by hp_run(S2)
 * equals hp_run(S1+S2) bit for bit. */
typedef struct {
    uint8_t *v;                     /* device [sum N_f * B] current assignment, 0/1     */
    void *nu;                       /* device [sum N_f * B] variance EMA: double for
                                       HP_FP64, float for HP_FP32                       */
    int32_t *s_max;                 /* device [F*B] best satisfied-clause count         */
    uint8_t *best;                  /* device [sum N_f * B] assignment achieving s_max  */
    int64_t *t;                     /* device [1] absolute sweep counter                */
    int64_t total_vars;             /* sum N_f the buffers were sized for (checked)     */
    int32_t n_formulas;             /* F the buffers were sized for (checked)           */
    int32_t chains;                 /* B the buffers were sized for (checked)           */
    int32_t nu_bytes;               /* sizeof(*nu): 4 for HP_FP32, else 8 (checked)     */
} hp_state;

typedef struct hp_plan_s *hp_plan_t;

/* Build a plan (formula-RBM assembly, Sec. 3.1 and eq. 4): validates the
 * batch, copies every host array, uploads the packed clause table, the
 * per-variable occurrence lists and the per-temperature tables, and enqueues
 * the table preparation on `stream`.  The plan owns its device memory until
 * hp_free.  Errors (HP_EINVAL, nothing allocated): K outside 1..7, L outside
 * 1..8 or rbm->k != cnf->k, N_f < 1 or C_f < 1, a literal with |lit| > N_f,
 * an all-zero clause, non-finite weights, alpha outside [0,1], chains < 1, a
 * temperature index outside [0, n_temps).  HP_EUNSUPPORTED: N_f > 32768, or
 * a formula whose working set exceeds the workgroup's LDS (160 KB on gfx950:
 * the push kernels take 9 bytes per variable plus their tables, which covers
 * N_f up to about 17 200; beyond that the pull kernel needs about
 * 20 KB + N_f + C_f bytes). */
hp_status hp_plan(hp_plan_t *out, const hp_cnf *cnf, const hp_rbm *rbm,
                  const hp_opts *opts, void *stream);

/* Enqueue n_sweeps >= 0 block-Gibbs rounds on every chain of every formula
 * (the inner loop of Sec. 3.2; 500 rounds per dispatch in the appendix
 * "Batching operations").  Each round first counts the satisfied clauses of
 * the current assignment and, on a strict improvement, records it in s_max
 * and best; n_sweeps = 0 performs only that count-and-track step.  *t is
 * advanced by n_sweeps.  HP_EINVAL if the state does not match the plan.
 * Runs of one plan must not overlap in time (a split launch uses the plan's
 * exchange buffers): issue them on one stream or order them with events. */
hp_status hp_run(hp_plan_t plan, const hp_state *state, int64_t n_sweeps, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sweeps as hp_run, bit for bit, but the run's scratch -- the persistent
 * launches' work counters and, for a split plan, the exchange mailboxes
 * between the workgroups of a chain -- comes from a static device array of
 * the library (16 MiB, held on every device the library has planned on until
 * the process ends) instead of the plan's buffers.  The call allocates
 * nothing: no hipMalloc, no graph instantiation (a plan built with graph = 1
 * launches directly here).  The state, the plan's tables and the plan's
 * time-out flag (hp_check) are used as in hp_run.  HP_EUNSUPPORTED if the
 * run needs more than 16 MiB of scratch (4 KiB of work counters plus, for a
 * split plan, about items * (8 G + 1) * N_max bytes of mailboxes); the
 * other errors are hp_run's.  Every call on one device shares that device's
 * array, which keeps the last call's contents (each call clears what must
 * start at zero): calls that overlap in time on one device -- on different
 * streams, or concurrent with another plan's hp_run_noalloc -- race and
 * their results are undefined; order them on one stream. */
hp_status hp_run_noalloc(hp_plan_t plan, const hp_state *state, int64_t n_sweeps, void *stream);

/* Autotuner: for every launch of the plan, time each candidate shape on
 * `n_sweeps` sweeps of the given state and keep the fastest.  A shape is a
 * workgroup size (64..1024), for the push kernels of the padded model in
 * FP64/FP32 the table layout (every table in LDS, the merged-padding words
 * of the contribution rows in global memory, or all contribution rows in
 * global memory: smaller LDS footprints let more workgroups share a CU), and
 * how a chain's waves share its clause steps (from a counter or dealt
 * round-robin).  All shapes compute the same bits.  The trial runs overwrite the state's v, nu, s_max and best
 * without advancing t, so pass a scratch state of the right shape.
 * Synchronous.  Cached graphs are discarded. */
hp_status hp_tune(hp_plan_t plan, const hp_state *scratch, int64_t n_sweeps, void *stream);

/* How a plan runs (for reports and tuning). */
typedef struct {
    int32_t threads;                /* largest workgroup size of any launch           */
    int32_t split;                  /* workgroups per chain of the push launch        */
    int32_t push_items;             /* (formula, chain) items on the push kernels     */
    int32_t pull_items;             /* (formula, chain) items on the pull kernel      */
    int32_t fx_shift;               /* S: push accumulators count units of 2^-S       */
    int32_t n_buckets;              /* launches per run (one per size class, push and
                                       pull formulas apart)                           */
    int64_t lds_push, lds_pull;     /* largest dynamic LDS bytes per workgroup        */
    /* first 16 launches: variant (0 push, 1 push with the contribution rows
     * in global memory, 2 pull, 3 push with the merged-padding words in
     * global memory), work items, workgroup size, largest N, persistent grid
     * (0 = one workgroup per item), clause-phase steps taken from a counter
     * (1) or dealt round-robin (0) */
    int32_t bucket_kind[16], bucket_items[16], bucket_threads[16], bucket_max_n[16], bucket_grid[16];
    int32_t bucket_dyn[16];
    int32_t forked;                 /* a plan of several launches: 1 = forked over side
                                       streams (some launch has one workgroup per item
                                       and may leave CUs free), 0 = in sequence on the
                                       caller's stream (every launch a persistent grid
                                       that fills the GPU)                            */
} hp_plan_info;

/* Fill *out with the plan's launch configuration.  HP_EINVAL on NULL. */
hp_status hp_plan_query(hp_plan_t plan, hp_plan_info *out);

/* Wait for the plan's device work and report device-side failures: returns
 * HP_EDEVICE if, since the plan was built or hp_check last returned, a
 * workgroup of a split launch (several workgroups per chain, hp_opts.split)
 * gave up waiting for the data of the others, in which case the state
 * written by those runs is void; HP_OK otherwise.  The failure flag is
 * sticky until this call reports it (later runs of the plan give up at once
 * while it is raised) and is cleared by the call. */
hp_status hp_check(hp_plan_t plan);

/* Release a plan's device memory (synchronises the device first).  NULL is
 * accepted. */
hp_status hp_free(hp_plan_t plan);

/* Checksum of the sweeps' random stream, for comparing the generator of two
 * builds and for timing it alone.  out[j] (j < n_out) is the XOR of all four
 * words of Philox4x32-10 (Salmon et al., SC'11) over the blocks
 * i = j * blocks .. (j + 1) * blocks - 1 at counter (t mod 2^32, chain,
 * phase * 2^31 + i, t div 2^32) with key (seed mod 2^32, (seed div 2^32) xor
 * formula) -- the counters and key a sweep of that chain uses, evaluated in
 * the sweep kernels' form (the first two rounds from per-sweep constants, two
 * blocks interleaved).  out: DEVICE [n_out] uint32.  HP_EINVAL unless
 * phase is 0 or 1, blocks >= 1, n_out >= 1 and (n_out * blocks) <= 2^31.
 * Stream-ordered. */
hp_status hp_philox_xor(uint64_t seed, int32_t formula, int64_t t, int32_t chain, int32_t phase, int64_t blocks,
                        int64_t n_out, uint32_t *out, void *stream);

/* Static description of a status code. */
const char *hp_status_string(hp_status s);

/* Message for the last failing call on this thread ("" if none). */
const char *hp_last_error(void);

/* ------------------------------------------------------------------------
 * Learned initial assignments.  The paper notes that learned components that
 * generate good initial assignments can be combined with the sampler
 * (Sec. 2); here a 32 -> 256 -> 1 perceptron maps per-variable occurrence
 * statistics of a formula to q_i = P(v_i = 1), is trained on labels produced
 * by the sampler itself, and seeds chains with v_i ~ Bernoulli(q_i); the
 * remaining chains keep their own (uniform) start, so the plain method stays
 * the fallback and the exact clause count judges the two.
 * ------------------------------------------------------------------------ */
#define HP_MLP_IN 32
#define HP_MLP_HIDDEN 256
/* parameter vector: W1 [32][256] | b1 [256] | w2 [256] | b2 [1] */
#define HP_MLP_PARAMS (HP_MLP_IN * HP_MLP_HIDDEN + 2 * HP_MLP_HIDDEN + 1)
/* rows of the backward pass's partial-sum workspace (one per workgroup) */
#define HP_MLP_PARTS 1024

typedef struct {                    /* caller-owned DEVICE buffers                     */
    float *params;                  /* [HP_MLP_PARAMS] FP32 master parameters          */
    float *adam_m, *adam_v;         /* [HP_MLP_PARAMS] Adam moments                    */
    float *grad;                    /* [HP_MLP_PARAMS] gradient of the mean loss       */
    uint16_t *w_bf16;               /* [32*256 + 256] bfloat16 copies: W1 transposed
                                       ([256][32]) then w2; refreshed by
                                       hp_mlp_sync and hp_mlp_adam                     */
    float *partials;                /* [HP_MLP_PARTS][HP_MLP_PARAMS + 1] workspace of
                                       hp_mlp_backward (its contents are scratch)      */
} hp_mlp;

/* Per-variable features of every formula of the plan, as bfloat16
 * [sum N_f][32] rows in variable order (layout of the counts: see the
 * kernels).  The plan allocates a small FP32 workspace on first use. */
hp_status hp_features(hp_plan_t plan, uint16_t *x, void *stream);

/* Refresh net->w_bf16 from net->params. */
hp_status hp_mlp_sync(const hp_mlp *net, void *stream);

/* q[r] = sigmoid(w2 . relu(W1^T x_r + b1) + b2) for rows r < rows (bfloat16
 * weights and inputs on MFMA, FP32 accumulation). */
hp_status hp_mlp_forward(const hp_mlp *net, const uint16_t *x, int64_t rows, float *q, void *stream);

/* net->grad = gradient of the mean binary cross-entropy of q against the
 * labels y in [0,1]; *loss_sum (device float) = the summed loss.  Each
 * workgroup writes the sums of its rows to its row of net->partials, and a
 * second kernel adds the rows up in a fixed order: for a given input the
 * gradient and the loss are the same bits on every call (no atomics).
 * Calls that share one partials buffer must not overlap. */
hp_status hp_mlp_backward(const hp_mlp *net, const uint16_t *x, const float *y, int64_t rows,
                          float *loss_sum, void *stream);

/* One Adam step (Kingma & Ba) on net->params with net->grad; step >= 1. */
hp_status hp_mlp_adam(const hp_mlp *net, float lr, float beta1, float beta2, float eps, int64_t step,
                      void *stream);

/* For chains chain_lo <= b < chain_hi of every formula: v[b][i] = [U < q_i]
 * with U drawn by the sweep generator at the reserved time 2^64 - 1
 * (visible phase, unit i).  q: device [sum N_f] in variable order. */
hp_status hp_init_chains(hp_plan_t plan, const float *q, int32_t chain_lo, int32_t chain_hi,
                         const hp_state *state, void *stream);

/* out[i] = mean over the chains of a [B][N_f]-layout byte array (for
 * example state->best): device [sum N_f] floats in variable order. */
hp_status hp_chain_mean(hp_plan_t plan, const uint8_t *a, float *out, void *stream);

/* ---- Prioritized unit propagation and the exchange (Sec. 3.4) ------------
 * Sec. 3.4 improves sampled assignments on the CPU: the floor(N/2) variables
 * with the highest variance average nu keep their sampled values and the
 * others are recomputed by unit propagation; the appendix program sends
 * (v, nu) to the host periodically and, some sweeps later, stacks the
 * returned assignments under the current ones and keeps the best B. */

/* Host.  New assignments of n_chains chains of formula `formula`:
 * v, out: HOST [n_chains][N_f] bytes (0/1); nu: HOST [n_chains][N_f] doubles.
 * Per chain: variables ordered by nu descending (ties by index); the first
 * floor(N/2) keep their values; every clause is examined once in clause
 * order (a clause with no true literal and one unassigned literal makes it
 * true; with none unassigned it is a conflict and stays unsatisfied); then
 * FIFO propagation (a dequeued variable re-examines, in clause order, the
 * clauses where its literal is false); then each remaining variable in
 * priority order that is still unassigned takes its sampled value and is
 * propagated.  A clause is the set of its distinct literals; 0 entries are
 * the clause's first literal.  threads: host threads (0 = all cores),
 * chains are independent.  Allocates host memory only; no GPU call. */
hp_status hp_unit_propagate(const hp_cnf *cnf, int32_t formula, int32_t n_chains, const uint8_t *v,
                            const double *nu, uint8_t *out, int32_t threads);

/* Device.  For every formula: counts the clauses satisfied by the current
 * state->v and by cand_v (DEVICE, the state's [sum N_f * B] layout), stacks
 * the 2B rows (current first), sorts the counts stably in ascending order
 * and keeps the last B rows as the new state->v (equal counts favour the
 * returned rows); a kept row takes the nu of the chain it came from.
 * s_max, best and t are unchanged.  The plan allocates its staging buffers
 * on first use.  Stream-ordered; cand_v must stay valid until it is done. */
hp_status hp_merge_candidates(hp_plan_t plan, const hp_state *state, const uint8_t *cand_v, void *stream);

/* ---- Replica exchange across the temperatures -----------------------------
 * Chains at temperature tau sample p_tau(v) ~ exp(-F_tau(v)), F_tau the
 * formula free energy (eq. 5: sum over clauses of the clause free energy,
 * eq. 1, of the clause's literal values, eq. 4).  One round, for every
 * formula: the pairs (tau, tau+1) with tau of the given parity pair the k-th
 * chain (by chain index) at tau with the k-th chain at tau + 1; a pair (a, b)
 * exchanges temperatures iff U < exp(min(D, 0)),
 *   D = F_tau(v_a) + F_tau+1(v_b) - F_tau(v_b) - F_tau+1(v_a),
 * U = (w >> 8) 2^-24, w = word 0 of the sweep generator's Philox at counter
 * (t mod 2^32, a, 2^31 - 1, t div 2^32) with t = *state->t (device).  The
 * plan's temperature of every (formula, chain) changes; v, nu, s_max, best
 * and t do not.  Up to 16 temperatures.  The plan allocates its workspace on
 * first use.  Stream-ordered. */
hp_status hp_temper(hp_plan_t plan, const hp_state *state, int32_t parity, void *stream);

/* Copies the plan's temperatures, HOST [n_formulas][chains] int32, and waits
 * for the copy on `stream`. */
hp_status hp_get_temps(hp_plan_t plan, int32_t *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HP_H */
