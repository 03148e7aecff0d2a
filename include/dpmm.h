/*
 * dpmm.h -- C ABI of libdpmm, an MI355X (gfx950) sampler for a
 * Dirichlet-process mixture of multinomials over single-cell UMI counts with
 * sub-cluster split/merge moves (Duan, Pinto & Xie, "Parallel Clustering of
 * Single Cell Transcriptomic Data with Split-Merge Sampling on Dirichlet
 * Process Mixtures", arXiv:1812.10048).
 *
 * Conventions for every entry point
 *   - Pointers are plain host or device addresses, as stated per argument.
 *     Device pointers must come from the GPU the context was created on.
 *   - Every call returns a dpmm_status.  The library never aborts or exits.
 *     On failure, dpmm_last_error() returns a message for the calling thread
 *     (valid until that thread's next call into the library).
 *   - A context is used by one host thread at a time.  Work is issued on the
 *     HIP stream given at init (a hipStream_t passed as void*, NULL meaning
 *     the default stream).  Calls marked "async" only enqueue work; calls
 *     marked "sync" wait for the stream before returning.
 *   - Paper notation: x_i^u is the UMI count of gene u in cell i, c_i the
 *     cluster of cell i and cbar_i in {0,1} its sub-cluster, theta_k and
 *     thetabar_{k,r} the multinomial parameters of clusters and sub-clusters,
 *     pi the mixing proportions, alpha the CRP parameter and lambda the
 *     Dirichlet hyper-parameter (here beta_u, one per gene, with
 *     lambdabar = lambda).
 */
#ifndef DPMM_H
#define DPMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dpmm_status {
    DPMM_OK = 0,
    DPMM_ERR_ARG = -1,          /* invalid argument (null pointer, size, range)    */
    DPMM_ERR_HIP = -2,          /* a HIP runtime call failed; message has its text  */
    DPMM_ERR_NOMEM = -3,        /* the workspace is smaller than required           */
    DPMM_ERR_STATE = -4,        /* context not usable for this call                 */
    DPMM_ERR_UNSUPPORTED = -5,  /* valid input outside what the library supports   */
    DPMM_ERR_DATA = -6          /* the CSR content failed validation on the device  */
} dpmm_status;

/* Arithmetic of the per-cell log-likelihood contraction (steps of Section 2.1
 * eq. 4 third line and Section 2.3 eq. 8).  Parameters are always redrawn in
 * FP64 and the split/merge ratios are always FP64. */
typedef enum dpmm_precision {
    DPMM_FP64 = 0,        /* FP64 log theta, FP64 accumulation                     */
    DPMM_FP32 = 1,        /* FP32 log theta, FP32 accumulation (vector ALU)        */
    DPMM_SPLIT_BF16 = 2   /* log theta = hi + lo in BF16, counts in BF16 (exact up
                             to 256, larger counts corrected in FP32), MFMA with
                             FP32 accumulation                                     */
} dpmm_precision;

/* UMI count matrix (Section 2.1: the V x N matrix x_i^u), given cell-major
 * as CSR.  All three arrays are DEVICE pointers, read only during dpmm_init
 * (the library keeps its own packed copy in the workspace), never written.
 * Columns must be strictly increasing within a row and < n_genes; values
 * must be in [1, 65535].  Violations make dpmm_init return DPMM_ERR_DATA. */
typedef struct dpmm_csr {
    int64_t n_cells;          /* N, >= 1                                           */
    int32_t n_genes;          /* G (the paper's V), 1 <= G <= 65535                */
    int32_t reserved;         /* must be 0                                         */
    int64_t nnz;              /* row_ptr[N]                                        */
    const int64_t* row_ptr;   /* device, N + 1 entries, row_ptr[0] = 0             */
    const int32_t* col;       /* device, nnz gene indices                          */
    const int32_t* val;       /* device, nnz counts                                */
} dpmm_csr;

/* dpmm_params.flags.  DPMM_FLAG_SPLIT_Q: the split ratio carries the
 * proposal term of Section 2.3.  A split proposes the current sub-clusters,
 * drawn with the eq. 8 probabilities p(cbar_i) of the last sweep, and the
 * reverse merge is certain, so log R gains -sum_{i in k} log p(cbar_i).
 * Without the flag the ratio is the collapsed one alone.  The per-cell
 * log p(cbar_i) are kept from the last sweep (8 bytes per cell of workspace),
 * are 0 for a cluster that re-drew its sub-labels at random, and are 0 after
 * dpmm_init and dpmm_set_state. */
#define DPMM_FLAG_SPLIT_Q 1u
/* DPMM_FLAG_NEW_CLUSTER: every sweep's Gibbs step runs over K + 1 clusters
 * (eq. 4).  Cluster K is appended empty, so its theta is drawn from the prior
 * Dir(beta) and its weight is the alpha component of pi ~ Dir(n_1..n_K,
 * alpha); it re-draws its sub-labels at random, and compaction drops it again
 * if no cell chose it.  Nothing is appended when K = k_max.  Without the flag
 * new clusters arise from splits only. */
#define DPMM_FLAG_NEW_CLUSTER 2u
/* DPMM_FLAG_RANDOM_SPLIT: a split/merge call runs a sub-cluster split pass, a
 * random-split pass or a merge pass, each with probability 1/3 (without the
 * flag: split or merge, 1/2 each).  A random split (chain B of Section 2.4)
 * halves every cluster by a fair Philox coin per cell; its ratio is the
 * collapsed split ratio of the two halves plus (n - 2) log 2, the reverse of
 * the eq. 23 merge.  An accepted cluster splits along the coins and both parts
 * re-draw their sub-labels.  dpmm_get_hastings reports the pass as 2.  Costs
 * one extra byte per cell and 16 k_max G bytes of workspace. */
#define DPMM_FLAG_RANDOM_SPLIT 4u
/* The moves as Sections 2.1-2.4 state them: the split ratio with its
 * Section 2.3 proposal term, the Gibbs step over K + 1 clusters of eq. 4, and
 * chain B's random splits beside the eq. 23 merge.  This is the recommended
 * setting; flags = 0 keeps the collapsed split ratio alone.  Neither setting
 * has the exact posterior as its stationary distribution on a handful of
 * cells (parallel passes, clusters emptied by the parallel sweep, and a
 * sub-cluster split whose reverse cannot be computed). */
#define DPMM_FLAGS_PAPER (DPMM_FLAG_SPLIT_Q | DPMM_FLAG_NEW_CLUSTER | DPMM_FLAG_RANDOM_SPLIT)

/* Hyper-parameters and sampler settings, copied at dpmm_init. */
typedef struct dpmm_params {
    double alpha;                  /* CRP parameter alpha (Section 2.1), > 0      */
    double beta;                   /* Dirichlet lambda for every gene, > 0, used
                                      when beta_per_gene is NULL                  */
    const double* beta_per_gene;   /* DEVICE, G entries > 0, or NULL; copied     */
    uint64_t seed;                 /* key of every Philox4x32-10 draw            */
    int32_t k_init;                /* initial clusters, 1..k_max (cells spread
                                      uniformly when > 1)                         */
    int32_t k_max;                 /* cluster capacity, 1..1024                   */
    int32_t precision;             /* dpmm_precision                               */
    uint32_t flags;                /* DPMM_FLAG_SPLIT_Q | DPMM_FLAG_NEW_CLUSTER |
                                      DPMM_FLAG_RANDOM_SPLIT                      */
    double refine_tol;             /* FP32 and split-BF16 only.  A cluster
                                      decision whose Gumbel gap is within the
                                      certified rounding bound of its two best
                                      scores is always re-scored in FP64; a
                                      value > 0 also re-scores decisions whose
                                      relative margin (top1 - top2) /
                                      max(1, |top1|) is below it.  <= 0: the
                                      bound alone                                  */
} dpmm_params;

typedef struct dpmm_ctx dpmm_ctx;

/* Counters of a context (cumulative since init or the last dpmm_set_state). */
typedef struct dpmm_stats_out {
    int64_t step;               /* Philox step: sweeps + split/merge calls so far */
    int32_t K;                  /* current number of clusters                     */
    int32_t last_pass;          /* -1 none yet, 0 split pass, 1 merge pass         */
    int64_t sweeps;
    int64_t sm_calls;
    int64_t splits_proposed;
    int64_t splits_accepted;
    int64_t merges_proposed;
    int64_t merges_accepted;
    int64_t kmax_skips;         /* accepted splits dropped for lack of capacity   */
    int64_t refined;            /* decisions re-scored in FP64                    */
    int64_t gamma_caps;         /* Gamma draws that hit the rejection cap (64)    */
    int64_t evals;              /* cell x cluster log-likelihood evaluations:
                                   the sum over sweeps of N (K + 2)              */
    int64_t near_tie;           /* cluster decisions whose FP64 relative Gumbel-max
                                   margin (top1 - top2) / max(1, |top1|) was
                                   below 1e-6 (always taken in FP64)             */
    double log_joint;           /* log p(c) + sum_k logDM(s_k) of the current
                                   partition (eq. 10 with Gamma(alpha) restored,
                                   eq. 12 integrated against eq. 28, multinomial
                                   coefficients dropped as in eq. 26), FP64     */
} dpmm_stats_out;

/* Stages of a sweep, a split/merge call and an empirical-Bayes step, for
 * dpmm_timing_stages. */
enum {
    DPMM_STAGE_REDRAW = 0,       /* a1 + a8: pi, theta, thetabar and the BF16 tables   */
    DPMM_STAGE_ASSIGN = 1,       /* a2 + a3: cluster log-likelihoods and draws         */
    DPMM_STAGE_REFINE = 2,       /* a3: FP64 re-score of uncertain decisions           */
    DPMM_STAGE_SUBCLUSTER = 3,   /* a3 + a4: sort by cluster, sub-cluster draws, stats  */
    DPMM_STAGE_COMPACT = 4,      /* empty clusters dropped, labels rewritten           */
    DPMM_STAGE_SPLIT_MERGE = 5,  /* a5: ratios, decisions, relabelling                 */
    DPMM_STAGE_EB = 6,           /* a6 + a7: empirical-Bayes beta step                 */
    DPMM_STAGE_LAYOUT = 7,       /* split-BF16: every 8th sweep, the check (and, when
                                    the partition changed, the rebuild) of the
                                    cluster-sorted copy of the counts              */
    DPMM_NUM_STAGES = 8
};

/* Message of the last failed call on this thread ("" if none). */
const char* dpmm_last_error(void);

/* Bytes of device workspace dpmm_init needs for this matrix and these
 * settings.  Pure host computation: reads only the sizes in csr and params. */
dpmm_status dpmm_workspace_size(const dpmm_csr* csr, const dpmm_params* params, size_t* bytes);

/* Create a sampler.  `workspace` is a DEVICE buffer of at least
 * dpmm_workspace_size() bytes, 256-byte aligned, owned by the caller, which
 * must keep it alive and untouched until dpmm_destroy.  Validates and packs
 * the CSR, draws the initial labels (all cells in one cluster, or spread over
 * k_init clusters), computes the sufficient statistics and flags every
 * cluster for a random sub-cluster start.  Sync.  On success *out owns a
 * small host object released by dpmm_destroy. */
dpmm_status dpmm_init(const dpmm_csr* csr, const dpmm_params* params, void* workspace,
                      size_t workspace_bytes, void* stream, dpmm_ctx** out);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): dpmm_init without the
 * workspace argument and without any allocation.  The workspace comes from a
 * static device array of 64 MiB that the library holds on every GPU it runs
 * on until the process ends (its last 256 bytes hold the launch hint that
 * dpmm_init keeps in pinned host memory), and the host context from a static
 * slot per device.  Matrices whose dpmm_workspace_size exceeds 64 MiB - 256
 * bytes are rejected with DPMM_ERR_NOMEM.  One such context per GPU at a
 * time: a second call before dpmm_destroy of the first returns
 * DPMM_ERR_STATE; calls on contexts that share the storage would race.  The
 * storage keeps the last context's contents; this call initialises every
 * part of it that the sampler reads.  Everything else is as dpmm_init
 * (inputs, stream, results: the same chain draw for draw).  Sync. */
dpmm_status dpmm_init_static(const dpmm_csr* csr, const dpmm_params* params, void* stream, dpmm_ctx** out);

/* Release the host object.  The workspace is the caller's to free afterwards
 * (after the stream has drained).  Sync. */
dpmm_status dpmm_destroy(dpmm_ctx* ctx);

/* n_sweeps sweeps of the instantiated sampler.  Each sweep:
 *   (a1) redraws pi ~ Dir(n_1..n_K, alpha), theta_k ~ Dir(lambda + s_k) and
 *        thetabar_{k,r} ~ Dir(lambda + s_{k,r})  (Section 2.1 eq. 4, first two
 *        lines; Section 2.3 eq. 19), in FP64;
 *   (a2-a3) draws every c_i by Gumbel-max over log pi_k + x_i . log theta_k
 *        (eq. 4 third line with eq. 26), then cbar_i within the chosen cluster
 *        with weights nbar_{k,r} less the cell's own old membership times
 *        prod_u thetabar^x (eq. 8); cells are independent given the parameters
 *        (Section 2.2);
 *   (a4) recomputes the integer statistics n_{k,r} and s_{k,r,u};
 *   then drops empty clusters and flags clusters with an empty sub-cluster
 *   for a random sub-cluster restart.  Async. */
dpmm_status dpmm_sweep(dpmm_ctx* ctx, int32_t n_sweeps);

/* One split/merge move (Sections 2.3-2.4, eq. 7).  A fair Philox coin picks
 * the split chain or the random-split/merge chain (Section 2.4, last
 * paragraph).  Split pass: every cluster whose sub-clusters are both
 * non-empty proposes the split into its sub-clusters with the collapsed
 * ratio log R = log alpha + lgamma(n_0) + lgamma(n_1) - lgamma(n)
 * + logDM(s_0) + logDM(s_1) - logDM(s) (eq. 10 with eq. 12 integrated over
 * theta).  Merge pass: every pair proposes the merge with the inverse ratio
 * times (1/2)^(n_1 + n_2 - 2) (eq. 23); accepted pairs are applied in random
 * order, each cluster at most once.  All ratios are FP64 lgamma sums.  Async. */
dpmm_status dpmm_split_merge(dpmm_ctx* ctx);

/* One empirical-Bayes fixed-point step for the per-gene lambda (beta_u), not
 * in the paper: beta_u <- beta_u * sum_k [psi(s_ku + beta_u) - psi(beta_u)]
 * / sum_k [psi(S_k + B) - psi(B)] over the current clusters (Minka 2000),
 * clamped to [1e-6, 1e6].  Async. */
dpmm_status dpmm_eb_update(dpmm_ctx* ctx);

/* Counters and the log joint into *out (HOST).  If nsub_host is not NULL it receives 2K int64
 * entries n_{k,r} at 2k + r (HOST, capacity 2 k_max).  If ssub_dev is not
 * NULL it receives the 2K x G int64 statistics s_{k,r,u} at (2k + r) G + u
 * (DEVICE, capacity 2 k_max G).  Sync. */
dpmm_status dpmm_stats(dpmm_ctx* ctx, dpmm_stats_out* out, int64_t* nsub_host, int64_t* ssub_dev);

/* Copy the labels c (int32) and cbar (uint8), N entries each, into DEVICE
 * buffers.  Sync. */
dpmm_status dpmm_get_labels(dpmm_ctx* ctx, int32_t* c_dev, uint8_t* cs_dev);

/* Replace the chain state: step counter, K, labels (DEVICE, N entries, c in
 * [0, K), cbar in {0,1}) and the K reset flags (HOST).  Statistics are
 * recomputed from the labels, counters are cleared.  Resuming from a saved
 * (step, K, c, cbar, reset, beta) reproduces the chain exactly.  Sync. */
dpmm_status dpmm_set_state(dpmm_ctx* ctx, int64_t step, int32_t K, const int32_t* c_dev,
                           const uint8_t* cs_dev, const uint8_t* reset_host);

/* The K reset flags (1 = the cluster re-draws its sub-labels at random on
 * the next sweep) into a HOST buffer of capacity k_max.  Sync. */
dpmm_status dpmm_get_reset_flags(dpmm_ctx* ctx, uint8_t* reset_host);

/* Parameters drawn by the last sweep, FP64 DEVICE buffers: log pi (k_max
 * entries, first K valid) and log theta (3 k_max x G: row k for cluster k,
 * row k_max + 2k + r for sub-cluster r of cluster k).  Sync. */
dpmm_status dpmm_get_params(dpmm_ctx* ctx, double* logpi_dev, double* logtheta_dev);

/* Per-gene lambda (beta_u), G FP64 entries, DEVICE buffers.  Sync. */
dpmm_status dpmm_get_beta(dpmm_ctx* ctx, double* beta_dev);
dpmm_status dpmm_set_beta(dpmm_ctx* ctx, const double* beta_dev);

/* Split/merge ratios of the last dpmm_split_merge: *pass (0 split, 1 merge,
 * -1 none), *n candidates, and, when not NULL, their FP64 log R (HOST, NaN
 * for clusters not eligible to split) and accept flags (HOST).  Split
 * candidate k is cluster k; merge candidate k2 (k2 - 1) / 2 + k1 is the pair
 * k1 < k2.  Capacity k_max + k_max (k_max - 1) / 2.  Sync. */
dpmm_status dpmm_get_hastings(dpmm_ctx* ctx, int32_t* pass, int32_t* n, double* logr_host,
                              uint8_t* accept_host);

/* Debug output of the sweep's own log-likelihood arithmetic: while set, every
 * sweep writes, per cell i, x_i . log theta_k for k < K followed by the two
 * sub-clusters of the cell's new cluster into a DEVICE buffer of
 * N x (k_cap + 2) entries (row stride k_cap + 2; requires K <= k_cap),
 * FP32 (fp64 = 0) or FP64 (fp64 = 1) elements.  The values are the ones the
 * decisions were taken on, before any FP64 re-scoring: FP64 for the FP64
 * precision, FP32 or split-BF16 accumulations otherwise; the two sub-cluster
 * scores are FP64 in every precision (NaN for a cluster that re-drew its
 * sub-labels at random).  NULL disables.  Sync. */
dpmm_status dpmm_set_debug_scores(dpmm_ctx* ctx, void* scores_dev, int32_t k_cap, int32_t fp64);

/* FP64 log-likelihoods of m listed cells against the parameters of the last
 * sweep's redraw (eq. 26, multinomial coefficient dropped): for the j-th
 * listed cell i, out[j (K + 2) + k] = x_i . log theta_k for k < K, then
 * x_i . log thetabar_{c_i,0} and x_i . log thetabar_{c_i,1} for its current
 * cluster c_i.  cells_dev: DEVICE int32[m], in [0, N); out_dev: DEVICE
 * FP64[m (K + 2)].  DPMM_ERR_STATE before the context's first sweep.
 * Sync. */
dpmm_status dpmm_dump_scores(dpmm_ctx* ctx, const int32_t* cells_dev, int32_t m, double* out_dev);

/* Split-BF16 tables of the last sweep (precision DPMM_SPLIT_BF16 only): the
 * bit patterns of hi = bf16(log theta) and lo = bf16(log theta - hi) for the
 * K clusters, K x G uint16 each, DEVICE.  Sync. */
dpmm_status dpmm_get_split_tables(dpmm_ctx* ctx, uint16_t* hi_dev, uint16_t* lo_dev);

/* Stage timing with HIP events on the context's stream.  While enabled,
 * every stage of a sweep, split/merge call and empirical-Bayes step (the
 * DPMM_STAGE_* list) is bracketed by an event pair (up to 16384 intervals
 * between two reads).  dpmm_timing_stages fills stage_ms and stage_count
 * (HOST, DPMM_NUM_STAGES entries each) with the summed milliseconds and the
 * number of intervals per stage since the last read, and resets them (sync);
 * dpmm_timing_read does the same for DPMM_STAGE_ASSIGN alone. */
dpmm_status dpmm_timing_enable(dpmm_ctx* ctx, int32_t enable);
dpmm_status dpmm_timing_stages(dpmm_ctx* ctx, double* stage_ms, int64_t* stage_count);
dpmm_status dpmm_timing_read(dpmm_ctx* ctx, double* total_ms, int64_t* launches);

/* Log Dirichlet-multinomial marginal of J count vectors (the per-cluster
 * factor of eq. 12 with theta integrated against eq. 28, without the
 * multinomial coefficient that eq. 26 drops):
 *   out[j] = lgamma(B) - lgamma(B + S_j) + sum_u [lgamma(beta_u + s_ju) - lgamma(beta_u)],
 * B = sum_u beta_u, S_j = sum_u s_ju.  s: J x G int64 (row-major, >= 0),
 * beta: G FP64 (> 0), out: J FP64; all DEVICE.  Stateless.  Async on stream. */
dpmm_status dpmm_dm_logmarginal(const int64_t* s, int32_t J, int32_t G, const double* beta,
                                double* out, void* stream);

/* Gradient of sum_j g_j out[j] with respect to beta:
 *   grad_beta[u] = sum_j g_j [psi(B) - psi(B + S_j) + psi(beta_u + s_ju) - psi(beta_u)].
 * s: J x G int64, beta: G, g: J, grad_beta: G FP64; all DEVICE.  Stateless.
 * Async on stream. */
dpmm_status dpmm_dm_grad(const int64_t* s, int32_t J, int32_t G, const double* beta,
                         const double* g, double* grad_beta, void* stream);

/* Preprocessing (Section 3 keeps the genes of largest standard deviation
 * across cells).  Exact per-gene moments of a cell-major CSR:
 *   sum[u] = sum_i x_iu,  sumsq[u] = sum_i x_iu^2,
 * as uint64 (no rounding; x <= 65535 and N < 2^30 keep both below 2^63).
 * sum_dev, sumsq_dev: DEVICE, G entries, overwritten.  Entries with a gene
 * outside [0, G) or a count < 1 are skipped (dpmm_init rejects such data).
 * The CSR is not otherwise validated.  Stateless; async on stream. */
dpmm_status dpmm_gene_moments(const dpmm_csr* csr, uint64_t* sum_dev, uint64_t* sumsq_dev, void* stream);

/* The k genes of largest standard deviation across the N cells (Section 3
 * keeps such genes), from the moments of dpmm_gene_moments.  The population
 * variance of gene u is B_u / N^2 with B_u = N sumsq[u] - sum[u]^2, formed
 * exactly in 128-bit integers, so the ranking is exact; equal B_u go to the
 * lower gene.
 *   sum_dev, sumsq_dev: DEVICE uint64[G] (dpmm_gene_moments of n_cells cells);
 *   map_dev: DEVICE int32[G], overwritten: the place of u among the chosen
 *     genes in increasing gene order, or -1 (the map dpmm_filter_genes takes);
 *   std_dev: DEVICE double[G] or NULL: sqrt(B_u) / N;
 *   k >= 0 (k >= G keeps every gene).
 * Stateless; async on stream. */
dpmm_status dpmm_top_genes(const uint64_t* sum_dev, const uint64_t* sumsq_dev, int32_t n_genes, int64_t n_cells,
                           int32_t k, int32_t* map_dev, double* std_dev, void* stream);

/* The CSR restricted to the genes u with map[u] >= 0, renumbered to map[u]
 * (map: DEVICE int32[G]; its kept values must increase with u, so that the
 * rows stay sorted, and lie in [0, G_out)).  Two calls:
 *   1. col_out == NULL: row_ptr_out (DEVICE, N + 1 entries) receives the new
 *      row offsets and *nnz_out (HOST) the new number of entries; this call
 *      synchronises the stream;
 *   2. col_out, val_out (DEVICE, *nnz_out entries each): the entries, in their
 *      row order; row_ptr_out must hold the offsets of call 1.
 * The caller owns every buffer. */
dpmm_status dpmm_filter_genes(const dpmm_csr* csr, const int32_t* map_dev, int64_t* row_ptr_out,
                              int32_t* col_out, int32_t* val_out, int64_t* nnz_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DPMM_H */
