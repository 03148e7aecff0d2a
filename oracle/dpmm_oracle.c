/*
 * dpmm_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, double-precision CPU implementation of the sub-cluster
 * split/merge sampler for a Dirichlet-process mixture of multinomials, as
 * described in Duan, Pinto & Xie, "Parallel Clustering of Single Cell
 * Transcriptomic Data with Split-Merge Sampling on Dirichlet Process
 * Mixtures" (arXiv:1812.10048).  It exists only so that the tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU library
 * against something obviously correct.  It shares no source with the GPU
 * library: its Philox generator, Gamma sampler, digamma, reductions and
 * relabelling are written here independently.
 *
 * Paper notation used below:
 *   x_i^u   UMI count of gene u in cell i         (Section 2.1, Table of notation)
 *   c_i     cluster of cell i; cbar_i in {0,1} its sub-cluster (Section 2.3)
 *   theta_k multinomial parameters of cluster k; thetabar_{k,r} of its sub-clusters
 *   pi      mixing proportions; alpha the CRP parameter; lambda (here beta_u,
 *           one per gene) the Dirichlet hyper-parameter; lambdabar = lambda.
 *   n_k, nbar_{k,r}  cell counts; s_{k,r,u} = sum of x_i^u over cells in (k,r).
 *
 * Readings of the paper that are not spelled out there (each is listed in the
 * design notes of the repository):
 *   - the split/merge ratios use the collapsed form obtained by integrating the
 *     Dirichlet prior (eq. 28) against the likelihood (eq. 12) and keeping the
 *     partition prior of eq. 10 with Gamma(alpha) restored;
 *   - the sub-cluster Gibbs step (eq. 8) uses the counts frozen at the start of
 *     the sweep, minus the cell's own old membership;
 *   - one move chain is chosen per split/merge call by a fair coin (Section 2.4);
 *   - ORACLE_EXACT: a chain built from the same pieces whose stationary
 *     distribution over partitions is exactly p(c | x): sweeps that would empty
 *     a cluster are undone, and each split/merge call makes one atomic chain-B
 *     move whose ratio carries its own proposal probabilities.  The tests
 *     check it by enumerating every partition of five and six cells.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared -o liboracle_dpmm.so dpmm_oracle.c -lm
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).        */
/* A counter-based generator, so that every draw is addressed by what it is  */
/* for: (element, sub-index, step, stream).                                 */
/* ------------------------------------------------------------------------ */

enum {
    ST_INIT = 1,      /* initial labels                                  */
    ST_GAMMA = 2,     /* Gamma variates for theta and thetabar            */
    ST_PI = 3,        /* Gamma variates for the mixing proportions        */
    ST_GUMBEL_C = 4,  /* Gumbel noise, cluster choice                     */
    ST_GUMBEL_S = 5,  /* Gumbel noise, sub-cluster choice                 */
    ST_RESUB = 6,     /* random sub-cluster labels of a reset cluster     */
    ST_CHAIN = 7,     /* which move chain a split/merge call runs         */
    ST_SPLIT = 8,     /* split acceptance uniforms                        */
    ST_MERGE = 9,     /* merge acceptance uniforms and visiting order     */
    ST_RSPLIT = 10    /* the per-cell coins of a random split             */
};

#define GAMMA_MAX_TRIES 64u

void oracle_philox4x32_10(uint32_t key0, uint32_t key1, const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t k0 = key0, k1 = key1;
    uint32_t a = ctr[0], b = ctr[1], c = ctr[2], d = ctr[3];
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)a;
        const uint64_t pc = (uint64_t)0xCD9E8D57u * (uint64_t)c;
        const uint32_t na = (uint32_t)(pc >> 32) ^ b ^ k0;
        const uint32_t nb = (uint32_t)pc;
        const uint32_t nc = (uint32_t)(pa >> 32) ^ d ^ k1;
        const uint32_t nd = (uint32_t)pa;
        a = na; b = nb; c = nc; d = nd;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = a; out[1] = b; out[2] = c; out[3] = d;
}

/* The four words addressed by (element, sub, step, stream, call). */
static void draw_words(uint64_t seed, uint32_t element, uint32_t sub, int64_t step,
                       uint32_t stream, uint32_t call, uint32_t w[4])
{
    uint32_t ctr[4];
    ctr[0] = element;
    ctr[1] = sub;
    ctr[2] = (uint32_t)step;
    ctr[3] = (stream << 24) | (call & 0xFFFFFFu);
    oracle_philox4x32_10((uint32_t)seed, (uint32_t)(seed >> 32), ctr, w);
}

/* 23 random bits -> odd multiple of 2^-24 in (0,1): exact in float and double. */
double oracle_u23(uint32_t w) { return ((double)(w >> 9) + 0.5) * 0x1p-23; }

/* 52 random bits -> odd multiple of 2^-53 in (0,1): exact in double. */
double oracle_u52(uint32_t hi, uint32_t lo)
{
    const uint64_t v = (((uint64_t)hi << 32) | (uint64_t)lo) >> 12;
    return ((double)v + 0.5) * 0x1p-52;
}

/* Standard Gumbel variate by inversion. */
static double gumbel(double u) { return -log(-log(u)); }

/* ------------------------------------------------------------------------ */
/* Special functions.                                                       */
/* ------------------------------------------------------------------------ */

double oracle_lgamma(double x)
{
    int sign;
    return lgamma_r(x, &sign);
}

/* Digamma for x > 0: shift up by psi(x) = psi(x+1) - 1/x until x >= 10, then
 * the asymptotic series of Abramowitz & Stegun 6.3.18 through z^-14. */
double oracle_digamma(double x)
{
    double shift = 0.0;
    while (x < 10.0) {
        shift -= 1.0 / x;
        x += 1.0;
    }
    const double r = 1.0 / x;
    const double r2 = r * r;
    const double tail =
        r2 * (1.0 / 12.0 -
        r2 * (1.0 / 120.0 -
        r2 * (1.0 / 252.0 -
        r2 * (1.0 / 240.0 -
        r2 * (1.0 / 132.0 -
        r2 * (691.0 / 32760.0 -
        r2 * (1.0 / 12.0)))))));
    return shift + log(x) - 0.5 * r - tail;
}

/* Neumaier-compensated running sum. */
typedef struct { double s, c; } ksum;
static inline void ksum_add(ksum* k, double v)
{
    const double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static inline double ksum_val(const ksum* k) { return k->s + k->c; }

/* ------------------------------------------------------------------------ */
/* Gamma variates (Marsaglia & Tsang, ACM TOMS 2000), returned as logs so   */
/* that tiny shapes cannot underflow.  Shape < 1 uses the boost            */
/* Gamma(a) = Gamma(a+1) * U^(1/a).  Normals come from Box-Muller.          */
/* Attempt j uses calls 2j (normal) and 2j+1 (acceptance and boost          */
/* uniforms) of the element's counter.                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t caps;        /* draws that hit the attempt cap                   */
    int64_t near_ties;   /* accept tests decided within 1e-12 (diagnostic)   */
} gamma_diag;

static double log_gamma_variate(double a, uint64_t seed, uint32_t element, uint32_t sub,
                                int64_t step, uint32_t stream, gamma_diag* diag)
{
    const int boost = a < 1.0;
    const double d = (boost ? a + 1.0 : a) - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    for (uint32_t j = 0; j < GAMMA_MAX_TRIES; ++j) {
        uint32_t w[4];
        draw_words(seed, element, sub, step, stream, 2u * j, w);
        const double u1 = oracle_u52(w[0], w[1]);
        const double u2 = oracle_u52(w[2], w[3]);
        const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        const double t = c * z;
        if (t <= -1.0) continue;           /* v = (1+t)^3 must be positive */
        uint32_t q[4];
        draw_words(seed, element, sub, step, stream, 2u * j + 1u, q);
        const double ua = oracle_u52(q[0], q[1]);
        /* log-acceptance 0.5 z^2 + d - d v + d log v, with v - 1 and log v
         * written through t to avoid cancellation for large d. */
        const double rhs = 0.5 * z * z + d * (3.0 * log1p(t) - t * (3.0 + t * (3.0 + t)));
        const double lhs = log(ua);
        if (diag && fabs(lhs - rhs) < 1e-12 * (1.0 + fabs(rhs))) diag->near_ties++;
        if (lhs < rhs) {
            double lg = log(d) + 3.0 * log1p(t);
            if (boost) lg += log(oracle_u52(q[2], q[3])) / a;
            return lg;
        }
    }
    if (diag) diag->caps++;
    return log(d);
}

double oracle_log_gamma_variate(double a, uint64_t seed, uint32_t element, uint32_t sub,
                                int64_t step, uint32_t stream)
{
    return log_gamma_variate(a, seed, element, sub, step, stream, NULL);
}

/* ------------------------------------------------------------------------ */
/* Model quantities.                                                        */
/* ------------------------------------------------------------------------ */

/* log of the Dirichlet-multinomial marginal of a count vector s (without the
 * multinomial coefficient, which the paper drops in eq. 26):  the integral of
 * prod_u theta_u^{s_u} against Dirichlet(theta | beta) (eq. 28), i.e. the
 * per-cluster factor of eq. 12 with theta integrated out:
 *   lgamma(B) - lgamma(B + S) + sum_u [lgamma(beta_u + s_u) - lgamma(beta_u)],
 * B = sum_u beta_u, S = sum_u s_u.  Terms with s_u = 0 vanish. */
double oracle_logdm(const int64_t* s, const double* beta, int32_t G)
{
    ksum acc = {0.0, 0.0};
    double B = 0.0;
    int64_t S = 0;
    for (int32_t u = 0; u < G; ++u) {
        B += beta[u];
        if (s[u] == 0) continue;
        S += s[u];
        ksum_add(&acc, oracle_lgamma(beta[u] + (double)s[u]));
        ksum_add(&acc, -oracle_lgamma(beta[u]));
    }
    ksum_add(&acc, oracle_lgamma(B));
    ksum_add(&acc, -oracle_lgamma(B + (double)S));
    return ksum_val(&acc);
}

/* log p(c) of eq. 10 (first equality) with the Gamma(alpha) factor that the
 * normaliser of Dir(n_1..n_K, alpha) requires:
 *   K log alpha + lgamma(alpha) - lgamma(alpha + N) + sum_k lgamma(n_k). */
double oracle_log_partition_prior(const int64_t* n, int32_t K, double alpha)
{
    ksum acc = {0.0, 0.0};
    int64_t N = 0;
    for (int32_t k = 0; k < K; ++k) {
        N += n[k];
        ksum_add(&acc, oracle_lgamma((double)n[k]));
    }
    ksum_add(&acc, (double)K * log(alpha));
    ksum_add(&acc, oracle_lgamma(alpha));
    ksum_add(&acc, -oracle_lgamma(alpha + (double)N));
    return ksum_val(&acc);
}

/* Gradient of sum_j g_j logDM(s_j; beta) with respect to beta_u:
 *   sum_j g_j [psi(B) - psi(B + S_j) + psi(beta_u + s_ju) - psi(beta_u)]. */
void oracle_dm_grad(const int64_t* s, int32_t J, int32_t G, const double* beta,
                    const double* g, double* grad)
{
    double B = 0.0;
    for (int32_t u = 0; u < G; ++u) B += beta[u];
    double common = 0.0;
    for (int32_t j = 0; j < J; ++j) {
        int64_t S = 0;
        for (int32_t u = 0; u < G; ++u) S += s[(int64_t)j * G + u];
        common += g[j] * (oracle_digamma(B) - oracle_digamma(B + (double)S));
    }
    for (int32_t u = 0; u < G; ++u) {
        double acc = common;
        const double psi_b = oracle_digamma(beta[u]);
        for (int32_t j = 0; j < J; ++j) {
            const int64_t v = s[(int64_t)j * G + u];
            if (v != 0) acc += g[j] * (oracle_digamma(beta[u] + (double)v) - psi_b);
        }
        grad[u] = acc;
    }
}

void oracle_dm_logmarginal(const int64_t* s, int32_t J, int32_t G, const double* beta, double* out)
{
    for (int32_t j = 0; j < J; ++j) out[j] = oracle_logdm(s + (int64_t)j * G, beta, G);
}

/* ------------------------------------------------------------------------ */
/* Sampler state.  All arrays are owned by the caller.                      */
/* ------------------------------------------------------------------------ */

enum { ORACLE_SPLIT_Q = 1u, ORACLE_NEW_CLUSTER = 2u, ORACLE_RANDOM_SPLIT = 4u, ORACLE_EXACT = 8u };

enum {
    CNT_GAMMA_CAPS = 0,
    CNT_GAMMA_NEAR_TIES = 1,
    CNT_SPLITS_PROPOSED = 2,
    CNT_SPLITS_ACCEPTED = 3,
    CNT_MERGES_PROPOSED = 4,
    CNT_MERGES_ACCEPTED = 5,
    CNT_KMAX_SKIPS = 6,
    CNT_SWEEPS = 7,
    CNT_SM_CALLS = 8,
    CNT_SWEEP_REVERTS = 9,
    N_COUNTERS = 16
};

typedef struct {
    /* data: cell-major CSR of UMI counts, columns sorted within a row */
    int64_t n_cells;
    int32_t n_genes;
    int32_t k_max;
    const int64_t* row_ptr;
    const int32_t* col;
    const int32_t* val;
    /* hyper-parameters */
    double alpha;
    double* beta;             /* [G]; the empirical-Bayes step updates it     */
    uint64_t seed;
    /* chain state */
    int64_t step;
    int32_t K;
    uint32_t flags;           /* ORACLE_SPLIT_Q: the split ratio carries the
                                 proposal term of Section 2.3;
                                 ORACLE_NEW_CLUSTER: the sweep draws over K + 1
                                 clusters (eq. 4), the last one new;
                                 ORACLE_RANDOM_SPLIT: a third pass of random
                                 splits (Section 2.4, chain B);
                                 ORACLE_EXACT (alone): the exact chain, see
                                 exact_sweep_check and exact_split_merge     */
    int32_t* c;               /* [N]                                          */
    uint8_t* cs;              /* [N] sub-cluster labels                       */
    uint8_t* reset;           /* [k_max] sub-labels to be re-drawn at random  */
    int64_t* nsub;            /* [2 k_max]   n of (k, r) at 2k + r            */
    int64_t* ssub;            /* [2 k_max G] counts of (k, r, u)              */
    double* logpi;            /* [k_max]                                      */
    double* logtheta;         /* [3 k_max G] rows k (clusters), then
                                 k_max + 2k + r (sub-clusters)                */
    /* diagnostics of the last sweep / split-merge call */
    double* margin_c;         /* [N] relative Gumbel-max margin, cluster      */
    double* margin_s;         /* [N] relative Gumbel-max margin, sub-cluster  */
    double* lpsub;            /* [N] log p(cbar_i) of eq. 8 in the last sweep
                                 (0 for a reset cluster or before any sweep)  */
    double* sm_logr;          /* [k_max + k_max (k_max - 1) / 2] log ratios   */
    double* sm_scale;         /* same size: sum of |terms| of each ratio      */
    uint8_t* sm_accept;       /* same size: 1 if accepted                     */
    int32_t sm_pass;          /* 0 split pass, 1 merge pass, 2 random splits  */
    int32_t sm_n;             /* number of candidates of the last call        */
    int32_t has_new;          /* 1 while cluster K - 1 is the new cluster of
                                 the current sweep (ORACLE_NEW_CLUSTER)       */
    int32_t pad2_;
    int64_t counters[N_COUNTERS];
} oracle_state;

static inline int64_t row_begin(const oracle_state* st, int64_t i) { return st->row_ptr[i]; }
static inline int64_t row_end(const oracle_state* st, int64_t i) { return st->row_ptr[i + 1]; }

/* Sufficient statistics: nbar_{k,r} and s_{k,r,u} from the labels. */
void oracle_stats(oracle_state* st)
{
    const int32_t G = st->n_genes;
    memset(st->nsub, 0, sizeof(int64_t) * 2 * (size_t)st->k_max);
    memset(st->ssub, 0, sizeof(int64_t) * 2 * (size_t)st->k_max * (size_t)G);
    for (int64_t i = 0; i < st->n_cells; ++i) {
        const int64_t grp = 2 * (int64_t)st->c[i] + st->cs[i];
        st->nsub[grp] += 1;
        int64_t* srow = st->ssub + grp * G;
        for (int64_t e = row_begin(st, i); e < row_end(st, i); ++e) srow[st->col[e]] += st->val[e];
    }
}

/* Remove empty clusters, keeping the order of the others; relabel cells and
 * move statistics and reset flags with them. */
static void compact(oracle_state* st)
{
    const int32_t G = st->n_genes;
    const int32_t K = st->K;
    int32_t* map = (int32_t*)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
    int32_t nk = 0;
    for (int32_t k = 0; k < K; ++k) {
        const int64_t n = st->nsub[2 * k] + st->nsub[2 * k + 1];
        map[k] = n > 0 ? nk++ : -1;
    }
    for (int32_t k = 0; k < K; ++k) {
        const int32_t j = map[k];
        if (j < 0 || j == k) continue;
        for (int r = 0; r < 2; ++r) {
            st->nsub[2 * j + r] = st->nsub[2 * k + r];
            memcpy(st->ssub + (int64_t)(2 * j + r) * G, st->ssub + (int64_t)(2 * k + r) * G,
                   sizeof(int64_t) * (size_t)G);
        }
        st->reset[j] = st->reset[k];
    }
    for (int32_t k = nk; k < K; ++k) {
        st->nsub[2 * k] = st->nsub[2 * k + 1] = 0;
        memset(st->ssub + (int64_t)2 * k * G, 0, sizeof(int64_t) * 2 * (size_t)G);
        st->reset[k] = 0;
    }
    for (int64_t i = 0; i < st->n_cells; ++i) st->c[i] = map[st->c[i]];
    st->K = nk;
    free(map);
}

/* Initial state: K = k_init clusters drawn uniformly (or one cluster), all
 * sub-labels 0 and every cluster flagged to re-draw its sub-labels. */
void oracle_init(oracle_state* st, int32_t k_init)
{
    for (int64_t i = 0; i < st->n_cells; ++i) {
        if (k_init <= 1) {
            st->c[i] = 0;
        } else {
            uint32_t w[4];
            draw_words(st->seed, (uint32_t)i, 0u, 0, ST_INIT, 0u, w);
            st->c[i] = (int32_t)(((uint64_t)w[0] * (uint64_t)k_init) >> 32);
        }
        st->cs[i] = 0;
    }
    st->K = k_init <= 1 ? 1 : k_init;
    memset(st->lpsub, 0, sizeof(double) * (size_t)st->n_cells);
    memset(st->reset, 0, (size_t)st->k_max);
    for (int32_t k = 0; k < st->K; ++k) st->reset[k] = 1;
    st->step = 0;
    st->has_new = 0;
    memset(st->counters, 0, sizeof(st->counters));
    oracle_stats(st);
    compact(st);
}

/* Set a state from labels (used to start both implementations from the same
 * point): statistics are recomputed from the labels. */
void oracle_set_state(oracle_state* st, int64_t step, int32_t K)
{
    st->step = step;
    st->K = K;
    st->has_new = 0;
    memset(st->lpsub, 0, sizeof(double) * (size_t)st->n_cells);
    oracle_stats(st);
}

/* ---- Step a1: parameter redraw (eq. 4, first two lines; eq. 19) ---------- */
/* pi ~ Dir(n_1, ..., n_K, alpha) (eq. 4 with eq. 10's posterior),
 * theta_k ~ Dir(beta + s_k), s_k = s_{k,0} + s_{k,1}   (eq. 4, second line),
 * thetabar_{k,r} ~ Dir(beta + s_{k,r})                (eq. 19, lambdabar = lambda).
 * Each Dirichlet is a vector of independent Gamma(shape_u, 1) variates
 * normalised to sum one; everything is kept as logarithms. */
static void dirichlet_row(oracle_state* st, int32_t row_id, const double* shape, int32_t n,
                          uint32_t stream, double* out, gamma_diag* diag)
{
    double m = -INFINITY;
    for (int32_t u = 0; u < n; ++u) {
        out[u] = log_gamma_variate(shape[u], st->seed, (uint32_t)u, (uint32_t)row_id, st->step,
                                   stream, diag);
        if (out[u] > m) m = out[u];
    }
    double tot = 0.0;
    for (int32_t u = 0; u < n; ++u) tot += exp(out[u] - m);
    const double lse = m + log(tot);
    for (int32_t u = 0; u < n; ++u) out[u] -= lse;
}

#define SUB_ROW_BASE 0x10000u

void oracle_redraw(oracle_state* st)
{
    const int32_t G = st->n_genes;
    const int32_t K = st->K;
    gamma_diag diag = {0, 0};

    /* mixing proportions: K cluster weights plus the alpha component; with a
     * new cluster in the sweep (eq. 4 over K + 1), the alpha component is its
     * weight pi_{K+1} */
    {
        const int32_t Kc = st->has_new ? K - 1 : K;     /* clusters with cells */
        double lg_alpha;
        double m = -INFINITY, tot = 0.0;
        for (int32_t k = 0; k < Kc; ++k) {
            const double n = (double)(st->nsub[2 * k] + st->nsub[2 * k + 1]);
            st->logpi[k] = log_gamma_variate(n, st->seed, (uint32_t)k, 0u, st->step, ST_PI, &diag);
            if (st->logpi[k] > m) m = st->logpi[k];
        }
        lg_alpha = log_gamma_variate(st->alpha, st->seed, 0xFFFFFFFFu, 0u, st->step, ST_PI, &diag);
        if (lg_alpha > m) m = lg_alpha;
        for (int32_t k = 0; k < Kc; ++k) tot += exp(st->logpi[k] - m);
        tot += exp(lg_alpha - m);
        const double lse = m + log(tot);
        for (int32_t k = 0; k < Kc; ++k) st->logpi[k] -= lse;
        if (st->has_new) st->logpi[Kc] = lg_alpha - lse;
    }

    const int32_t nrows = 3 * K;
    int64_t caps = 0, ties = 0;
#pragma omp parallel reduction(+ : caps, ties)
    {
        double* shape = (double*)malloc(sizeof(double) * (size_t)G);
        gamma_diag local = {0, 0};
#pragma omp for schedule(dynamic, 1)
        for (int32_t row = 0; row < nrows; ++row) {
            double* out;
            int32_t row_id;
            if (row < K) {
                const int32_t k = row;
                const int64_t* s0 = st->ssub + (int64_t)(2 * k) * G;
                const int64_t* s1 = s0 + G;
                for (int32_t u = 0; u < G; ++u) shape[u] = st->beta[u] + (double)(s0[u] + s1[u]);
                out = st->logtheta + (int64_t)k * G;
                row_id = k;
            } else {
                const int32_t q = row - K;      /* q = 2k + r */
                const int64_t* sr = st->ssub + (int64_t)q * G;
                for (int32_t u = 0; u < G; ++u) shape[u] = st->beta[u] + (double)sr[u];
                out = st->logtheta + (int64_t)(st->k_max + q) * G;
                row_id = (int32_t)(SUB_ROW_BASE + (uint32_t)q);
            }
            dirichlet_row(st, row_id, shape, G, ST_GAMMA, out, &local);
        }
        caps += local.caps;
        ties += local.near_ties;
        free(shape);
    }
    st->counters[CNT_GAMMA_CAPS] += caps + diag.caps;
    st->counters[CNT_GAMMA_NEAR_TIES] += ties + diag.near_ties;
}

/* ---- Steps a2-a3: log-likelihoods and Gumbel-max assignment --------------- */
/* c_i ~ pi_k prod_u theta_{k,u}^{x_i^u}  (eq. 4 third line, eq. 26), drawn as
 * argmax_k [log pi_k + sum_u x_i^u log theta_{k,u} + g_{ik}] with standard
 * Gumbel g.  Then, within the chosen cluster k (eq. 8),
 * cbar_i ~ nbar_{k,r,-i} prod_u thetabar_{k,r,u}^{x_i^u}, where nbar_{k,r,-i}
 * are the counts at the start of the sweep minus the cell's own old
 * membership.  If both are zero the two sub-clusters get equal weight.  A
 * cluster flagged for reset instead draws cbar_i as a fair coin. */

static double rel_margin(double top1, double top2)
{
    if (!(top2 > -INFINITY)) return INFINITY;
    return (top1 - top2) / fmax(1.0, fabs(top1));
}

/* loglik of cell i against one log-parameter row */
static double cell_loglik(const oracle_state* st, int64_t i, const double* logrow)
{
    double acc = 0.0;
    for (int64_t e = row_begin(st, i); e < row_end(st, i); ++e)
        acc += (double)st->val[e] * logrow[st->col[e]];
    return acc;
}

void oracle_assign(oracle_state* st)
{
    const int32_t G = st->n_genes;
    const int32_t K = st->K;
    const int64_t N = st->n_cells;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i) {
        const int32_t c_old = st->c[i];
        const int32_t s_old = st->cs[i];
        double top1 = -INFINITY, top2 = -INFINITY;
        int32_t best = 0;
        uint32_t w[4];
        for (int32_t k = 0; k < K; ++k) {
            if ((k & 3) == 0) draw_words(st->seed, (uint32_t)i, (uint32_t)(k >> 2), st->step, ST_GUMBEL_C, 0u, w);
            const double v = st->logpi[k] + cell_loglik(st, i, st->logtheta + (int64_t)k * G) +
                             gumbel(oracle_u23(w[k & 3]));
            if (v > top1) {
                top2 = top1;
                top1 = v;
                best = k;
            } else if (v > top2) {
                top2 = v;
            }
        }
        st->margin_c[i] = rel_margin(top1, top2);

        const int32_t k = best;
        int32_t sub;
        if (st->reset[k]) {
            draw_words(st->seed, (uint32_t)i, 0u, st->step, ST_RESUB, 0u, w);
            sub = (int32_t)(w[0] >> 31);
            st->margin_s[i] = INFINITY;
            st->lpsub[i] = 0.0;
        } else {
            int64_t wt[2];
            for (int r = 0; r < 2; ++r) wt[r] = st->nsub[2 * k + r] - ((c_old == k && s_old == r) ? 1 : 0);
            double lw[2];
            for (int r = 0; r < 2; ++r) {
                if (wt[0] == 0 && wt[1] == 0) lw[r] = 0.0;
                else lw[r] = wt[r] > 0 ? log((double)wt[r]) : -INFINITY;
            }
            draw_words(st->seed, (uint32_t)i, 0u, st->step, ST_GUMBEL_S, 0u, w);
            double ll[2], v[2];
            for (int r = 0; r < 2; ++r) {
                ll[r] = lw[r] + cell_loglik(st, i, st->logtheta + (int64_t)(st->k_max + 2 * k + r) * G);
                v[r] = ll[r] + gumbel(oracle_u23(w[r]));
            }
            sub = v[1] > v[0] ? 1 : 0;
            st->margin_s[i] = rel_margin(fmax(v[0], v[1]), fmin(v[0], v[1]));
            /* the eq. 8 probability of the drawn sub-label: a two-way softmax */
            const double m = fmax(ll[0], ll[1]);
            st->lpsub[i] = ll[sub] - (m + log(exp(ll[0] - m) + exp(ll[1] - m)));
        }
        st->c[i] = k;
        st->cs[i] = (uint8_t)sub;
    }
}

/* Clear the reset flags consumed by the sweep, drop emptied clusters, and flag
 * clusters of at least two cells with an empty sub-cluster for reset. */
static void finish_sweep(oracle_state* st)
{
    st->has_new = 0;
    memset(st->reset, 0, (size_t)st->k_max);
    compact(st);
    for (int32_t k = 0; k < st->K; ++k) {
        const int64_t n0 = st->nsub[2 * k], n1 = st->nsub[2 * k + 1];
        st->reset[k] = (n0 + n1 >= 2 && (n0 == 0 || n1 == 0)) ? 1 : 0;
    }
}

/* With ORACLE_NEW_CLUSTER the sweep's Gibbs step runs over K + 1 clusters
 * (eq. 4): cluster K is appended empty, so its theta is a draw from the prior
 * Dir(beta) and its weight is the alpha component of pi; it re-draws its
 * sub-labels at random like any new cluster, and compaction drops it again
 * if no cell chose it.  Nothing is appended at k_max. */
void oracle_extend(oracle_state* st)
{
    st->has_new = 0;
    if (!(st->flags & ORACLE_NEW_CLUSTER) || st->K >= st->k_max) return;
    const int32_t k = st->K;
    st->nsub[2 * k] = st->nsub[2 * k + 1] = 0;
    memset(st->ssub + (int64_t)(2 * k) * st->n_genes, 0, sizeof(int64_t) * 2 * (size_t)st->n_genes);
    st->reset[k] = 1;
    st->K = k + 1;
    st->has_new = 1;
}

/* ORACLE_EXACT, the sweep.  Given (pi, theta), the labels' exact conditional
 * under the joint p(c, x) p(pi | c) p(theta | c, x) is prod_i pi_{c_i}
 * f(x_i | theta_{c_i}) restricted to labelings that keep all K clusters
 * non-empty: the Dirichlet Dir(n_1..n_K, alpha) of eq. 4 has no density at a
 * zero count, so a labeling that empties a cluster has conditional
 * probability 0.  The cells' independent draws (Section 2.2) are then an
 * independence proposal from the unrestricted product, and its
 * Metropolis-Hastings acceptance is 1 when every cluster keeps a cell and 0
 * otherwise: such a sweep is undone as a whole.  Returns 1 if undone. */
static int exact_sweep_check(oracle_state* st, const int32_t* c_before, const uint8_t* cs_before)
{
    for (int32_t k = 0; k < st->K; ++k) {
        if (st->nsub[2 * k] + st->nsub[2 * k + 1] > 0) continue;
        memcpy(st->c, c_before, sizeof(int32_t) * (size_t)st->n_cells);
        memcpy(st->cs, cs_before, (size_t)st->n_cells);
        oracle_stats(st);
        st->counters[CNT_SWEEP_REVERTS] += 1;
        return 1;
    }
    return 0;
}

/* One sweep: redraw (a1), assign (a2-a3), statistics (a4), compaction. */
void oracle_sweep(oracle_state* st)
{
    const int exact = (st->flags & ORACLE_EXACT) != 0;
    int32_t* c_before = NULL;
    uint8_t* cs_before = NULL;
    oracle_extend(st);
    oracle_redraw(st);
    if (exact) {
        c_before = (int32_t*)malloc(sizeof(int32_t) * (size_t)(st->n_cells > 0 ? st->n_cells : 1));
        cs_before = (uint8_t*)malloc((size_t)(st->n_cells > 0 ? st->n_cells : 1));
        memcpy(c_before, st->c, sizeof(int32_t) * (size_t)st->n_cells);
        memcpy(cs_before, st->cs, (size_t)st->n_cells);
    }
    oracle_assign(st);
    oracle_stats(st);
    if (exact) {
        exact_sweep_check(st, c_before, cs_before);
        free(c_before);
        free(cs_before);
    }
    finish_sweep(st);
    st->counters[CNT_SWEEPS] += 1;
    st->step += 1;
}

/* Assignment only, from log-parameters already in the state (no redraw). */
void oracle_assign_only(oracle_state* st)
{
    oracle_assign(st);
}

/* ---- Step a5: split / merge Hastings ratios (eq. 7) ---------------------- */
/* Collapsed split ratio for cluster k with sub-clusters k0, k1 (the eq. 14
 * partition-prior part, in its collapsed eq. 10 form, times the eq. 16
 * theta/x part with theta integrated out):
 *   log R = log alpha + lgamma(nbar0) + lgamma(nbar1) - lgamma(n)
 *         + logDM(s0) + logDM(s1) - logDM(s0 + s1).
 * The merge of k1 < k2 is the reverse move of a random split (Section 2.4),
 * whose proposal ratio is (1/2)^(n1 + n2 - 2) (eq. 23):
 *   log R = -[log alpha + lgamma(n1) + lgamma(n2) - lgamma(n1 + n2)
 *             + logDM(s1) + logDM(s2) - logDM(s1 + s2)] + (n1 + n2 - 2) log 1/2.
 * The ratio and the sum of the magnitudes of its terms are returned. */
static double logdm_parts(const int64_t* a, const int64_t* b, const double* beta, int32_t G,
                          double* scale)
{
    /* logDM(a) + logDM(b) - logDM(a + b), with b = NULL meaning "a alone" */
    ksum acc = {0.0, 0.0};
    double B = 0.0, mag = 0.0;
    int64_t Sa = 0, Sb = 0;
    for (int32_t u = 0; u < G; ++u) {
        B += beta[u];
        const int64_t va = a[u], vb = b ? b[u] : 0;
        Sa += va;
        Sb += vb;
        if (va + vb == 0) continue;
        const double lb = oracle_lgamma(beta[u]);
        double t;
        if (va) { t = oracle_lgamma(beta[u] + (double)va) - lb; ksum_add(&acc, t); mag += fabs(t); }
        if (vb) { t = oracle_lgamma(beta[u] + (double)vb) - lb; ksum_add(&acc, t); mag += fabs(t); }
        if (b) { t = oracle_lgamma(beta[u] + (double)(va + vb)) - lb; ksum_add(&acc, -t); mag += fabs(t); }
    }
    double t;
    if (b) {
        const double lB = oracle_lgamma(B);
        t = lB - oracle_lgamma(B + (double)Sa); ksum_add(&acc, t); mag += fabs(t);
        t = lB - oracle_lgamma(B + (double)Sb); ksum_add(&acc, t); mag += fabs(t);
        t = lB - oracle_lgamma(B + (double)(Sa + Sb)); ksum_add(&acc, -t); mag += fabs(t);
    } else {
        t = oracle_lgamma(B) - oracle_lgamma(B + (double)Sa); ksum_add(&acc, t); mag += fabs(t);
    }
    if (scale) *scale = mag;
    return ksum_val(&acc);
}

double oracle_split_logr(const int64_t* s0, const int64_t* s1, int64_t n0, int64_t n1,
                         const double* beta, int32_t G, double alpha, double* scale)
{
    double mag;
    const double dm = logdm_parts(s0, s1, beta, G, &mag);
    const double prior = log(alpha) + oracle_lgamma((double)n0) + oracle_lgamma((double)n1) -
                         oracle_lgamma((double)(n0 + n1));
    if (scale) *scale = mag + fabs(log(alpha)) + fabs(oracle_lgamma((double)n0)) +
                        fabs(oracle_lgamma((double)n1)) + fabs(oracle_lgamma((double)(n0 + n1)));
    return prior + dm;
}

double oracle_merge_logr(const int64_t* s1, const int64_t* s2, int64_t n1, int64_t n2,
                         const double* beta, int32_t G, double alpha, double* scale)
{
    double sc;
    const double split = oracle_split_logr(s1, s2, n1, n2, beta, G, alpha, &sc);
    const double q = (double)(n1 + n2 - 2) * log(0.5);
    if (scale) *scale = sc + fabs(q);
    return -split + q;
}

static int64_t pair_index(int32_t k1, int32_t k2) { return (int64_t)k2 * (k2 - 1) / 2 + k1; }

typedef struct { uint64_t key; int64_t p; int32_t k1, k2; } merge_cand;
static int cmp_cand(const void* x, const void* y)
{
    const merge_cand* a = (const merge_cand*)x;
    const merge_cand* b = (const merge_cand*)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->p < b->p ? -1 : (a->p > b->p ? 1 : 0);
}

/* ORACLE_EXACT, the moves.  One atomic move per call (Section 2.4: atomic
 * moves picked at random), from chain B only: with probability 1/2 a random
 * split of one cluster k picked uniformly among the K, every cell of k taking
 * a fair Philox coin (stream RSPLIT), else a merge of one pair picked
 * uniformly among the K (K - 1) / 2.  A labelled split {A, B} of n cells
 * comes from two coin vectors, so its proposal probability is
 * (1/2) (1/K) 2^(1-n), and its reverse, the merge of A and B from K + 1
 * clusters, has (1/2) / C(K + 1, 2).  Eq. 7 with the collapsed joint (eq. 10
 * with Gamma(alpha) restored, eq. 12 integrated against eq. 28) then gives
 *   log R_split = logR_c(A, B) + n log 2 - log(K + 1),
 *   log R_merge = -logR_c(A, B) - n log 2 + log K   (K counted before),
 * logR_c the collapsed ratio of oracle_split_logr.  A coin vector with an
 * empty side, a split at k_max and a merge at K = 1 leave the state as it
 * is.  The candidate's ratio is reported as sm_logr[0] (NaN if none). */
static void exact_split_merge(oracle_state* st, double coin)
{
    const int32_t G = st->n_genes;
    const int32_t K = st->K;
    const int64_t N = st->n_cells;
    uint32_t q[4];
    draw_words(st->seed, 1u, 0u, st->step, ST_CHAIN, 0u, q);
    const double u_pick = oracle_u52(q[0], q[1]);
    const double u_acc = oracle_u52(q[2], q[3]);
    st->sm_n = 1;
    st->sm_logr[0] = NAN;
    st->sm_scale[0] = 0.0;
    st->sm_accept[0] = 0;
    if (coin < 0.5) {
        st->sm_pass = 2;
        const int32_t k = (int32_t)(u_pick * (double)K);
        int64_t hn[2] = {0, 0};
        int64_t* hs = (int64_t*)calloc(2 * (size_t)G, sizeof(int64_t));
        uint8_t* side = (uint8_t*)calloc((size_t)(N > 0 ? N : 1), 1);
        for (int64_t i = 0; i < N; ++i) {
            if (st->c[i] != k) continue;
            uint32_t cw[4];
            draw_words(st->seed, (uint32_t)i, 0u, st->step, ST_RSPLIT, 0u, cw);
            side[i] = (uint8_t)(cw[0] >> 31);
            hn[side[i]] += 1;
            for (int64_t e = row_begin(st, i); e < row_end(st, i); ++e) hs[side[i] * G + st->col[e]] += st->val[e];
        }
        if (hn[0] > 0 && hn[1] > 0 && K < st->k_max) {
            st->counters[CNT_SPLITS_PROPOSED] += 1;
            double sc;
            const double lr = oracle_split_logr(hs, hs + G, hn[0], hn[1], st->beta, G, st->alpha, &sc) +
                              (double)(hn[0] + hn[1]) * log(2.0) - log((double)(K + 1));
            st->sm_logr[0] = lr;
            st->sm_scale[0] = sc + (double)(hn[0] + hn[1]) * log(2.0) + log((double)(K + 1));
            if (log(u_acc) < lr) {
                for (int64_t i = 0; i < N; ++i)
                    if (st->c[i] == k && side[i]) st->c[i] = K;
                st->K = K + 1;
                st->reset[k] = 1;
                st->reset[K] = 1;
                st->sm_accept[0] = 1;
                st->counters[CNT_SPLITS_ACCEPTED] += 1;
            }
        }
        free(side);
        free(hs);
    } else {
        st->sm_pass = 1;
        if (K >= 2) {
            const int64_t npairs = (int64_t)K * (K - 1) / 2;
            const int64_t p = (int64_t)(u_pick * (double)npairs);
            int32_t k2 = 1;
            while ((int64_t)(k2 + 1) * k2 / 2 <= p) k2++;
            const int32_t k1 = (int32_t)(p - (int64_t)k2 * (k2 - 1) / 2);
            int64_t* sk = (int64_t*)calloc(2 * (size_t)G, sizeof(int64_t));
            for (int32_t u = 0; u < G; ++u) {
                sk[u] = st->ssub[(int64_t)(2 * k1) * G + u] + st->ssub[(int64_t)(2 * k1 + 1) * G + u];
                sk[G + u] = st->ssub[(int64_t)(2 * k2) * G + u] + st->ssub[(int64_t)(2 * k2 + 1) * G + u];
            }
            const int64_t n1 = st->nsub[2 * k1] + st->nsub[2 * k1 + 1];
            const int64_t n2 = st->nsub[2 * k2] + st->nsub[2 * k2 + 1];
            st->counters[CNT_MERGES_PROPOSED] += 1;
            double sc;
            const double lr = -oracle_split_logr(sk, sk + G, n1, n2, st->beta, G, st->alpha, &sc) -
                              (double)(n1 + n2) * log(2.0) + log((double)K);
            st->sm_logr[0] = lr;
            st->sm_scale[0] = sc + (double)(n1 + n2) * log(2.0) + log((double)K);
            if (log(u_acc) < lr) {
                /* as in the merge pass: the merged cluster's sub-clusters are
                 * its two parts */
                for (int64_t i = 0; i < N; ++i) {
                    if (st->c[i] == k1) st->cs[i] = 0;
                    else if (st->c[i] == k2) { st->c[i] = k1; st->cs[i] = 1; }
                }
                st->reset[k1] = 0;
                st->reset[k2] = 0;
                st->sm_accept[0] = 1;
                st->counters[CNT_MERGES_ACCEPTED] += 1;
            }
            free(sk);
        }
    }
    oracle_stats(st);
    compact(st);
}

void oracle_split_merge(oracle_state* st)
{
    const int32_t G = st->n_genes;
    const int32_t K = st->K;
    uint32_t w[4];
    draw_words(st->seed, 0u, 0u, st->step, ST_CHAIN, 0u, w);
    /* pass 0: split into the sub-clusters; 1: merges; 2: random splits (only
     * with ORACLE_RANDOM_SPLIT, the three then equally likely) */
    const double coin = oracle_u52(w[0], w[1]);
    if (st->flags & ORACLE_EXACT) {
        exact_split_merge(st, coin);
        st->counters[CNT_SM_CALLS] += 1;
        st->step += 1;
        return;
    }
    int pass;
    if (st->flags & ORACLE_RANDOM_SPLIT) pass = coin < 1.0 / 3.0 ? 0 : (coin < 2.0 / 3.0 ? 2 : 1);
    else pass = coin < 0.5 ? 0 : 1;
    const int split_pass = pass != 1;
    st->sm_pass = pass;

    int64_t* s_k = (int64_t*)malloc(sizeof(int64_t) * (size_t)(K > 0 ? K : 1) * (size_t)G);
    for (int32_t k = 0; k < K; ++k)
        for (int32_t u = 0; u < G; ++u)
            s_k[(int64_t)k * G + u] = st->ssub[(int64_t)(2 * k) * G + u] + st->ssub[(int64_t)(2 * k + 1) * G + u];

    if (split_pass) {
        st->sm_n = K;
        int32_t K_new = K;
        int32_t* newlab = (int32_t*)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
        /* The two halves of each cluster: its sub-clusters (pass 0), or
         * (pass 2, chain B of Section 2.4) a fair coin per cell, whose split is
         * the reverse of the eq. 23 merge: log R gains (n - 2) log 2. */
        const int64_t N = st->n_cells;
        int64_t* hn = st->nsub;
        int64_t* hs = st->ssub;
        uint8_t* side = NULL;
        if (pass == 2) {
            side = (uint8_t*)malloc((size_t)(N > 0 ? N : 1));
            hn = (int64_t*)calloc(2 * (size_t)(K > 0 ? K : 1), sizeof(int64_t));
            hs = (int64_t*)calloc(2 * (size_t)(K > 0 ? K : 1) * (size_t)G, sizeof(int64_t));
            for (int64_t i = 0; i < N; ++i) {
                uint32_t cw[4];
                draw_words(st->seed, (uint32_t)i, 0u, st->step, ST_RSPLIT, 0u, cw);
                side[i] = (uint8_t)(cw[0] >> 31);
                const int64_t h = 2 * (int64_t)st->c[i] + side[i];
                hn[h] += 1;
                for (int64_t e = row_begin(st, i); e < row_end(st, i); ++e) hs[h * G + st->col[e]] += st->val[e];
            }
        }
        /* Section 2.3: the split proposes the current sub-clusters, with
         * probability q = prod_{i in k} p(cbar_i) (eq. 8), and the reverse merge
         * is certain; with ORACLE_SPLIT_Q the ratio carries -Q_k = -log q. */
        double* Q = (double*)calloc((size_t)(K > 0 ? K : 1), sizeof(double));
        if (st->flags & ORACLE_SPLIT_Q)
            for (int64_t i = 0; i < st->n_cells; ++i) Q[st->c[i]] += st->lpsub[i];
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t k = 0; k < K; ++k) {
            const int64_t n0 = hn[2 * k], n1 = hn[2 * k + 1];
            if ((pass == 0 && st->reset[k]) || n0 < 1 || n1 < 1) {
                st->sm_logr[k] = NAN;
                st->sm_scale[k] = 0.0;
                continue;
            }
            const double extra = pass == 2 ? (double)(n0 + n1 - 2) * log(2.0) : -Q[k];
            st->sm_logr[k] = oracle_split_logr(hs + (int64_t)(2 * k) * G, hs + (int64_t)(2 * k + 1) * G,
                                               n0, n1, st->beta, G, st->alpha, &st->sm_scale[k]) +
                             extra;
            st->sm_scale[k] += fabs(extra);
        }
        free(Q);
        for (int32_t k = 0; k < K; ++k) {
            newlab[k] = -1;
            st->sm_accept[k] = 0;
            if (isnan(st->sm_logr[k])) continue;
            st->counters[CNT_SPLITS_PROPOSED] += 1;
            uint32_t q[4];
            draw_words(st->seed, (uint32_t)k, 0u, st->step, ST_SPLIT, 0u, q);
            if (log(oracle_u52(q[0], q[1])) < st->sm_logr[k]) {
                if (K_new < st->k_max) {
                    newlab[k] = K_new++;
                    st->sm_accept[k] = 1;
                    st->counters[CNT_SPLITS_ACCEPTED] += 1;
                } else {
                    st->counters[CNT_KMAX_SKIPS] += 1;
                }
            }
        }
        /* half 1 of each accepted cluster becomes the new cluster */
        for (int64_t i = 0; i < N; ++i) {
            const int32_t j = newlab[st->c[i]];
            if (j < 0) continue;
            if ((side ? side[i] : st->cs[i]) == 1) st->c[i] = j;
            st->cs[i] = 0;
        }
        for (int32_t k = 0; k < K; ++k) {
            const int32_t j = newlab[k];
            if (j < 0) continue;
            st->nsub[2 * j] = hn[2 * k + 1];
            st->nsub[2 * j + 1] = 0;
            st->nsub[2 * k] = hn[2 * k];
            st->nsub[2 * k + 1] = 0;
            memcpy(st->ssub + (int64_t)(2 * j) * G, hs + (int64_t)(2 * k + 1) * G, sizeof(int64_t) * (size_t)G);
            if (hs != st->ssub)
                memcpy(st->ssub + (int64_t)(2 * k) * G, hs + (int64_t)(2 * k) * G, sizeof(int64_t) * (size_t)G);
            memset(st->ssub + (int64_t)(2 * j + 1) * G, 0, sizeof(int64_t) * (size_t)G);
            memset(st->ssub + (int64_t)(2 * k + 1) * G, 0, sizeof(int64_t) * (size_t)G);
            st->reset[k] = 1;
            st->reset[j] = 1;
        }
        st->K = K_new;
        free(newlab);
        if (side) {
            free(side);
            free(hn);
            free(hs);
        }
    } else {
        const int64_t npairs = (int64_t)K * (K - 1) / 2;
        st->sm_n = (int32_t)npairs;
        merge_cand* cand = (merge_cand*)malloc(sizeof(merge_cand) * (size_t)(npairs > 0 ? npairs : 1));
        int64_t ncand = 0;
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t k2 = 1; k2 < K; ++k2) {
            for (int32_t k1 = 0; k1 < k2; ++k1) {
                const int64_t p = pair_index(k1, k2);
                const int64_t n1 = st->nsub[2 * k1] + st->nsub[2 * k1 + 1];
                const int64_t n2 = st->nsub[2 * k2] + st->nsub[2 * k2 + 1];
                st->sm_logr[p] = oracle_merge_logr(s_k + (int64_t)k1 * G, s_k + (int64_t)k2 * G, n1, n2,
                                                   st->beta, G, st->alpha, &st->sm_scale[p]);
            }
        }
        for (int32_t k2 = 1; k2 < K; ++k2) {
            for (int32_t k1 = 0; k1 < k2; ++k1) {
                const int64_t p = pair_index(k1, k2);
                st->sm_accept[p] = 0;
                st->counters[CNT_MERGES_PROPOSED] += 1;
                uint32_t q[4];
                draw_words(st->seed, (uint32_t)p, 0u, st->step, ST_MERGE, 0u, q);
                if (log(oracle_u52(q[0], q[1])) < st->sm_logr[p]) {
                    cand[ncand].key = ((uint64_t)q[2] << 32) | (uint64_t)q[3];
                    cand[ncand].p = p;
                    cand[ncand].k1 = k1;
                    cand[ncand].k2 = k2;
                    ncand++;
                }
            }
        }
        /* visit the accepted pairs in ascending random key; a cluster takes
         * part in at most one merge per call */
        qsort(cand, (size_t)ncand, sizeof(merge_cand), cmp_cand);
        int32_t* into = (int32_t*)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
        uint8_t* used = (uint8_t*)calloc((size_t)(K > 0 ? K : 1), 1);
        for (int32_t k = 0; k < K; ++k) into[k] = -1;
        for (int64_t q = 0; q < ncand; ++q) {
            const int32_t k1 = cand[q].k1, k2 = cand[q].k2;
            if (used[k1] || used[k2]) continue;
            used[k1] = used[k2] = 1;
            into[k2] = k1;
            into[k1] = k1;
            st->sm_accept[cand[q].p] = 1;
            st->counters[CNT_MERGES_ACCEPTED] += 1;
        }
        for (int64_t i = 0; i < st->n_cells; ++i) {
            const int32_t k = st->c[i];
            if (into[k] < 0) continue;
            st->cs[i] = (uint8_t)(into[k] != k);
            st->c[i] = into[k];
        }
        for (int32_t k2 = 0; k2 < K; ++k2) {
            const int32_t k1 = into[k2];
            if (k1 < 0 || k1 == k2) continue;
            st->nsub[2 * k1] = st->nsub[2 * k1] + st->nsub[2 * k1 + 1];
            st->nsub[2 * k1 + 1] = st->nsub[2 * k2] + st->nsub[2 * k2 + 1];
            st->nsub[2 * k2] = st->nsub[2 * k2 + 1] = 0;
            for (int32_t u = 0; u < G; ++u) {
                st->ssub[(int64_t)(2 * k1) * G + u] = s_k[(int64_t)k1 * G + u];
                st->ssub[(int64_t)(2 * k1 + 1) * G + u] = s_k[(int64_t)k2 * G + u];
                st->ssub[(int64_t)(2 * k2) * G + u] = 0;
                st->ssub[(int64_t)(2 * k2 + 1) * G + u] = 0;
            }
            st->reset[k1] = 0;
            st->reset[k2] = 0;
        }
        free(into);
        free(used);
        free(cand);
        compact(st);
    }
    free(s_k);
    st->counters[CNT_SM_CALLS] += 1;
    st->step += 1;
}

/* n iterations of (sweep, split/merge), for long chains on tiny data. */
void oracle_iterate(oracle_state* st, int64_t n)
{
    for (int64_t t = 0; t < n; ++t) {
        oracle_sweep(st);
        oracle_split_merge(st);
    }
}

/* ---- Steps a6-a7: empirical-Bayes update of the per-gene beta ----------- */
/* One fixed-point step (Minka 2000, "Estimating a Dirichlet distribution")
 * on sum_k logDM(s_k; beta) over the K clusters:
 *   beta_u <- beta_u * sum_k [psi(s_ku + beta_u) - psi(beta_u)]
 *                    / sum_k [psi(S_k + B) - psi(B)],
 * clamped to [1e-6, 1e6]. */
void oracle_eb_update(oracle_state* st)
{
    const int32_t G = st->n_genes;
    const int32_t K = st->K;
    double B = 0.0;
    for (int32_t u = 0; u < G; ++u) B += st->beta[u];
    double den = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        int64_t S = 0;
        for (int32_t u = 0; u < G; ++u)
            S += st->ssub[(int64_t)(2 * k) * G + u] + st->ssub[(int64_t)(2 * k + 1) * G + u];
        den += oracle_digamma((double)S + B) - oracle_digamma(B);
    }
    double* nb = (double*)malloc(sizeof(double) * (size_t)G);
#pragma omp parallel for schedule(static)
    for (int32_t u = 0; u < G; ++u) {
        const double b = st->beta[u];
        const double psi_b = oracle_digamma(b);
        double num = 0.0;
        for (int32_t k = 0; k < K; ++k) {
            const int64_t v = st->ssub[(int64_t)(2 * k) * G + u] + st->ssub[(int64_t)(2 * k + 1) * G + u];
            if (v) num += oracle_digamma((double)v + b) - psi_b;
        }
        double x = den > 0.0 ? b * num / den : b;
        nb[u] = fmin(1e6, fmax(1e-6, x));
    }
    memcpy(st->beta, nb, sizeof(double) * (size_t)G);
    free(nb);
}

/* Collapsed log joint log p(c) + sum_k logDM(s_k), up to the dropped
 * multinomial coefficients: a chain diagnostic. */
double oracle_log_joint(const oracle_state* st)
{
    const int32_t G = st->n_genes;
    const int32_t K = st->K;
    int64_t* n = (int64_t*)malloc(sizeof(int64_t) * (size_t)(K > 0 ? K : 1));
    int64_t* s = (int64_t*)malloc(sizeof(int64_t) * (size_t)G);
    ksum acc = {0.0, 0.0};
    for (int32_t k = 0; k < K; ++k) {
        n[k] = st->nsub[2 * k] + st->nsub[2 * k + 1];
        for (int32_t u = 0; u < G; ++u)
            s[u] = st->ssub[(int64_t)(2 * k) * G + u] + st->ssub[(int64_t)(2 * k + 1) * G + u];
        ksum_add(&acc, oracle_logdm(s, st->beta, G));
    }
    ksum_add(&acc, oracle_log_partition_prior(n, K, st->alpha));
    free(n);
    free(s);
    return ksum_val(&acc);
}

/* Log-likelihood dump for a sample of cells: for each listed cell i,
 * out[j][k] = sum_u x_i^u log theta_{k,u} (k < K), then the two
 * sub-clusters of the cell's current cluster at K and K + 1. */
void oracle_cell_logliks(const oracle_state* st, const int64_t* cells, int64_t m, double* out)
{
    const int32_t G = st->n_genes;
    const int32_t K = st->K;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) {
        const int64_t i = cells[j];
        double* o = out + j * (K + 2);
        for (int32_t k = 0; k < K; ++k) o[k] = cell_loglik(st, i, st->logtheta + (int64_t)k * G);
        const int32_t k = st->c[i];
        for (int r = 0; r < 2; ++r)
            o[K + r] = cell_loglik(st, i, st->logtheta + (int64_t)(st->k_max + 2 * k + r) * G);
    }
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
