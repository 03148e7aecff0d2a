// splitmerge.hip -- step a5: split/merge Hastings ratios (Section 2.3 eq. 7)
// in their collapsed form and the moves they accept.
//
// With logDM(s) = lgamma(B) - lgamma(B + S) + sum_u [lgamma(beta_u + s_u) -
// lgamma(beta_u)] (eq. 12 integrated over theta against the Dirichlet
// normaliser of eq. 28) and the partition prior of eq. 10 (with Gamma(alpha)),
//   split of k into its sub-clusters:
//     log R = log alpha + lgamma(n_0) + lgamma(n_1) - lgamma(n)
//           + logDM(s_0) + logDM(s_1) - logDM(s_0 + s_1)
//   merge of k1 < k2 (reverse of a random split, eq. 23):
//     log R = -[log alpha + lgamma(n_1) + lgamma(n_2) - lgamma(n_1 + n_2)
//             + logDM(s_1) + logDM(s_2) - logDM(s_1 + s_2)] + (n_1 + n_2 - 2) log 1/2.
// The per-gene sums are FP64 with compensated accumulation, over workgroups of
// (candidate, gene tile) combined in tile order; the decisions are taken by a
// single workgroup.
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

constexpr int kSmThreads = 512;          // split and cluster passes: K x gene-tile workgroups
constexpr int kMergeThreads = 256;       // merge pass: K (K - 1) / 2 workgroups

// Compensated accumulator (Neumaier): value = s + c.
struct CSum {
    double s = 0.0, c = 0.0;
    __device__ inline void add(double v)
    {
        const double t = s + v;
        c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
        s = t;
    }
    __device__ inline void merge(const CSum& o)
    {
        add(o.s);
        c += o.c;
    }
    __device__ inline double value() const { return s + c; }
};

// Workgroup reduction of a compensated sum, three int64 sums and a double.
struct SmRed {
    CSum cs;
    long long a, b;
    double beta;
};

template <int NT>
__device__ inline SmRed block_reduce(SmRed v)
{
    __shared__ double ls[NT], lc[NT], lb[NT];
    __shared__ long long la[NT], lbb[NT];
    const int t = threadIdx.x;
    ls[t] = v.cs.s; lc[t] = v.cs.c; la[t] = v.a; lbb[t] = v.b; lb[t] = v.beta;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (t < off) {
            CSum x; x.s = ls[t]; x.c = lc[t];
            CSum y; y.s = ls[t + off]; y.c = lc[t + off];
            x.merge(y);
            ls[t] = x.s; lc[t] = x.c;
            la[t] += la[t + off];
            lbb[t] += lbb[t + off];
            lb[t] += lb[t + off];
        }
        __syncthreads();
    }
    SmRed r;
    r.cs.s = ls[0]; r.cs.c = lc[0]; r.a = la[0]; r.b = lbb[0]; r.beta = lb[0];
    __syncthreads();
    return r;
}

// log Gamma(x) for x > 0, for the per-gene terms: Stirling's series with the
// Bernoulli-number terms through x^-7 once x >= 16 (the first omitted term,
// 1 / (1188 x^9), is below 1.2e-14 there), reached from a smaller x by the
// recurrence log Gamma(x) = log Gamma(x + m) - log(x (x + 1) ... (x + m - 1)).
__device__ inline double lgamma_pos(double x)
{
    double shift = 0.0;
    if (x < 16.0) {
        double p = 1.0;
        while (x < 16.0) {
            p *= x;
            x += 1.0;
        }
        shift = -log(p);
    }
    const double r = 1.0 / x, r2 = r * r;
    const double series = r * (1.0 / 12.0 - r2 * (1.0 / 360.0 - r2 * (1.0 / 1260.0 - r2 * (1.0 / 1680.0))));
    return (x - 0.5) * log(x) - x + 0.91893853320467274178 + series + shift;   // 0.5 log(2 pi)
}

// lgamma(beta_u + v) - lgamma(beta_u) of gene u, zero for v = 0
// (lgb = lgamma(beta_u)); small counts come from the gene's table, which
// holds the same expression evaluated by k_lgamma_beta
__device__ inline double rising(const Ws& ws, int u, double beta, double lgb, long long v)
{
    if ((unsigned long long)v < (unsigned long long)kRiseTab) return ws.lgrise[(int64_t)u * kRiseTab + v];
    return lgamma_pos(beta + (double)v) - lgb;
}

// One thread per (gene, v < kRiseTab): lgbeta and the gene's table.  Each
// thread evaluates lgamma(beta_u) itself (the same value in all of them).
__global__ void k_lgamma_beta(Ws ws)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)ws.G * kRiseTab) return;
    const int u = (int)(q / kRiseTab);
    const int v = (int)(q % kRiseTab);
    const double b = ws.beta[u];
    const double lgb = lgamma(b);
    if (v == 0) ws.lgbeta[u] = lgb;
    ws.lgrise[q] = v ? lgamma_pos(b + (double)v) - lgb : 0.0;
}

void launch_lgamma_beta(const Ws& ws, hipStream_t s)
{
    const int64_t n = (int64_t)ws.G * kRiseTab;
    hipLaunchKernelGGL(k_lgamma_beta, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ws);
}

// The split ratios and the clusters' logDM in two passes, so that K clusters
// spread over K x tiles workgroups: pass 1 reduces one tile of kSmThreads genes
// of one cluster (a compensated sum and the count and beta sums); pass 2
// combines a cluster's tiles in tile order and adds the per-cluster terms.
// mode 0: split into the sub-clusters (not for a reset cluster); 1: split
// into the coin halves held in ws.ssub / ws.nsub by the caller, with the
// (n - 2) log 2 that reverses the eq. 23 merge; 2: logDM(s_{k,0} + s_{k,1}).
static_assert(kSmGenes == kSmThreads, "one gene per thread of a tile");

__device__ inline bool split_eligible(unsigned long long n0, unsigned long long n1, uint8_t reset, int mode)
{
    return !((mode == 0 && reset) || n0 < 1 || n1 < 1);
}

// Workgroup (x, tile) takes clusters x, x + gridDim.x, ... below K (the grid
// is sized from a recent K): their counts, beta and log Gamma(beta) loaded
// together with what decides the cluster's eligibility.
__global__ void __launch_bounds__(kSmThreads) k_sm_tiles(Ws ws, int mode)
{
    const int K = ws.st->K;
    const int G = ws.G;
    const int T = gridDim.y;
    const int u = blockIdx.y * kSmThreads + threadIdx.x;
    for (int k = blockIdx.x; k < K; k += gridDim.x) {
        const unsigned long long* s0 = ws.ssub + (int64_t)(2 * k) * G;
        const unsigned long long* s1 = s0 + G;
        long long x0 = 0, x1 = 0;
        double bu = 0.0, lgb = 0.0;
        if (u < G) {
            x0 = (long long)s0[u];
            x1 = (long long)s1[u];
            bu = ws.beta[u];
            lgb = ws.lgbeta[u];
        }
        const unsigned long long n0 = ws.nsub[2 * k], n1 = ws.nsub[2 * k + 1];
        const uint8_t rst = ws.reset[k];
        if (mode != 2 && !split_eligible(n0, n1, rst, mode)) continue;
        SmRed r;
        r.a = r.b = 0;
        r.beta = 0.0;
        if (u < G) {
            r.beta = bu;
            if (mode == 2) {
                const long long v = x0 + x1;
                r.a = v;
                r.cs.add(rising(ws, u, bu, lgb, v));
            } else {
                r.a = x0;
                r.b = x1;
                if (x0 + x1 != 0) {
                    r.cs.add(rising(ws, u, bu, lgb, x0));
                    r.cs.add(rising(ws, u, bu, lgb, x1));
                    r.cs.add(-rising(ws, u, bu, lgb, x0 + x1));
                }
            }
        }
        r = block_reduce<kSmThreads>(r);
        if (threadIdx.x == 0) {
            SmPart& o = ws.sm_part[(int64_t)k * T + blockIdx.y];
            o.s = r.cs.s;
            o.c = r.cs.c;
            o.beta = r.beta;
            o.a = r.a;
            o.b = r.b;
        }
    }
}

// One wavefront per cluster: every lane sums the tiles' B and counts in tile
// order, lane j evaluates the j-th log-gamma term, and lane 0 adds them to the
// tiles' compensated sums in a fixed order.
__global__ void __launch_bounds__(64) k_sm_finish(Ws ws, int mode, int T)
{
    const int K = ws.st->K;
    const int lane = threadIdx.x;
    for (int k = blockIdx.x; k < K; k += gridDim.x) {
        const SmPart* part = ws.sm_part + (int64_t)k * T;
        const unsigned long long n0 = ws.nsub[2 * k], n1 = ws.nsub[2 * k + 1];
        if (mode != 2 && !split_eligible(n0, n1, ws.reset[k], mode)) {
            if (lane == 0) {
                ws.sm_logr[k] = __builtin_nan("");
                if (mode == 0) ws.qsub[k] = 0.0;        // ready for the next split pass
            }
            continue;
        }
        double B = 0.0;
        long long a = 0, b = 0;
#pragma unroll 8
        for (int q = 0; q < T; ++q) {
            B += part[q].beta;
            a += part[q].a;
            b += part[q].b;
        }
        // the argument per lane, then one log-gamma call shared by all lanes
        // (a different call per lane would run one after another)
        double arg = 1.0;
        switch (lane) {
        case 0: arg = B; break;
        case 1: arg = B + (double)a; break;
        case 2: arg = B + (double)b; break;
        case 3: arg = B + (double)(a + b); break;
        case 4: arg = (double)n0; break;
        case 5: arg = (double)n1; break;
        case 6: arg = (double)(n0 + n1); break;
        default: break;
        }
        double x = lgamma_pos(arg);
        if (lane == 7) x = log(ws.alpha);
        double lg[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) lg[j] = __shfl(x, j);
        if (lane == 0) {
            CSum tot;
            for (int q = 0; q < T; ++q) {
                CSum y;
                y.s = part[q].s;
                y.c = part[q].c;
                tot.merge(y);
            }
            tot.add(lg[0] - lg[1]);
            if (mode == 2) {
                ws.dm_k[k] = tot.value();
            } else {
                tot.add(lg[0] - lg[2]);
                tot.add(-(lg[0] - lg[3]));
                tot.add(lg[7] + lg[4] + lg[5] - lg[6]);
                if (mode == 1) tot.add((double)(n0 + n1 - 2) * log(2.0));    // chain B, Section 2.4
                else if (ws.flags & kFlagSplitQ) tot.add(-ws.qsub[k]);      // proposal term, Section 2.3
                if (mode == 0) ws.qsub[k] = 0.0;        // ready for the next split pass
                ws.sm_logr[k] = tot.value();
            }
        }
    }
}

// k_guess: a recent K (sizes the grids; the kernels loop over any K)
static int k_grid(const Ws& ws, int k_guess)
{
    return k_guess > 0 && k_guess < ws.k_max ? k_guess : ws.k_max;
}

static void launch_sm_pair(const Ws& ws, int mode, int k_guess, hipStream_t s)
{
    const int T = sm_tiles(ws.G);
    const int kb = k_grid(ws, k_guess);
    hipLaunchKernelGGL(k_sm_tiles, dim3((unsigned)kb, (unsigned)T), dim3(kSmThreads), 0, s, ws, mode);
    hipLaunchKernelGGL(k_sm_finish, dim3((unsigned)kb), dim3(64), 0, s, ws, mode, T);
}

// The collapsed log joint of the current partition (a chain diagnostic):
// log p(c) + sum_k logDM(s_k), with log p(c) = K log alpha + lgamma(alpha)
// - lgamma(alpha + N) + sum_k lgamma(n_k) (eq. 10 with Gamma(alpha) restored)
// and logDM(s_k) from the cluster pass (mode 2).  One thread, clusters in
// order, compensated.
__global__ void k_log_joint(Ws ws)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int K = ws.st->K;
    CSum tot;
    for (int k = 0; k < K; ++k) {
        tot.add(ws.dm_k[k]);
        tot.add(lgamma((double)(ws.nsub[2 * k] + ws.nsub[2 * k + 1])));
    }
    tot.add((double)K * log(ws.alpha));
    tot.add(lgamma(ws.alpha));
    tot.add(-lgamma(ws.alpha + (double)ws.N));
    ws.st->log_joint = tot.value();
}

void launch_log_joint(const Ws& ws, hipStream_t s)
{
    launch_sm_pair(ws, 2, ws.k_max, s);
    hipLaunchKernelGGL(k_log_joint, dim3(1), dim3(64), 0, s, ws);
}

__device__ inline void pair_of(long long p, int* k1, int* k2)
{
    int b = (int)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
    while ((long long)b * (b - 1) / 2 > p) --b;
    while ((long long)(b + 1) * b / 2 <= p) ++b;
    *k2 = b;
    *k1 = (int)(p - (long long)b * (b - 1) / 2);
}

__global__ void __launch_bounds__(kMergeThreads) k_merge_ratios(Ws ws)
{
    const int K = ws.st->K;
    const int G = ws.G;
    const long long npairs = (long long)K * (K - 1) / 2;
    for (long long p = blockIdx.x; p < npairs; p += gridDim.x) {
        int k1, k2;
        pair_of(p, &k1, &k2);
        const unsigned long long* a0 = ws.ssub + (int64_t)(2 * k1) * G;
        const unsigned long long* b0 = ws.ssub + (int64_t)(2 * k2) * G;
        SmRed r;
        r.a = r.b = 0;
        r.beta = 0.0;
        for (int u = threadIdx.x; u < G; u += kMergeThreads) {
            const double bu = ws.beta[u];
            const long long v = (long long)(a0[u] + a0[u + G] + b0[u] + b0[u + G]);
            r.beta += bu;
            r.a += v;
            r.cs.add(rising(ws, u, bu, ws.lgbeta[u], v));
        }
        r = block_reduce<kMergeThreads>(r);
        if (threadIdx.x < 64) {     // wavefront 0: one log-gamma term per lane, as in k_sm_finish
            const int lane = threadIdx.x;
            const double n1 = (double)(ws.nsub[2 * k1] + ws.nsub[2 * k1 + 1]);
            const double n2 = (double)(ws.nsub[2 * k2] + ws.nsub[2 * k2 + 1]);
            double arg = 1.0;
            switch (lane) {
            case 0: arg = n1; break;
            case 1: arg = n2; break;
            case 2: arg = n1 + n2; break;
            case 3: arg = r.beta; break;
            case 4: arg = r.beta + (double)r.a; break;
            default: break;
            }
            const double x = lgamma_pos(arg);
            double lg[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) lg[j] = __shfl(x, j);
            if (lane == 0) {
                CSum split;   // log R of splitting the union into k1 and k2
                split.add(log(ws.alpha) + lg[0] + lg[1] - lg[2]);
                split.add(ws.dm_k[k1]);
                split.add(ws.dm_k[k2]);
                CSum dm12 = r.cs;
                dm12.add(lg[3] - lg[4]);
                split.add(-dm12.s);
                split.add(-dm12.c);
                ws.sm_logr[p] = -split.value() + (n1 + n2 - 2.0) * log(0.5);
            }
        }
    }
}

// Q_k = sum over the cells now in cluster k of log p(cbar_i) from the last
// sweep (the split proposal term of Section 2.3), formed here from the score
// difference of each cell's draw and its sub-label (only split passes need
// it): per-workgroup LDS sums, then one FP64 atomic per cluster into qsub,
// which is zero on entry (k_sm_finish clears it after use).  Each thread takes
// kQCells cells a workgroup-width apart, all loads issued before the sums.
constexpr int kQThreads = 1024;
constexpr int kQCells = 4;
__global__ void __launch_bounds__(kQThreads) k_split_q(Ws ws, const int32_t* __restrict__ c,
                                                       const uint8_t* __restrict__ cs)
{
    extern __shared__ double qacc[];     // [K]
    const int64_t i0 = (int64_t)blockIdx.x * (kQThreads * kQCells) + threadIdx.x;
    int kk[kQCells];
    double dd[kQCells];
    int sb[kQCells];
#pragma unroll
    for (int j = 0; j < kQCells; ++j) {
        const int64_t i = i0 + (int64_t)j * kQThreads;
        const bool in = i < ws.N;
        kk[j] = in ? c[i] : -1;
        dd[j] = in ? ws.subdd[i] : __builtin_nan("");
        sb[j] = in ? (cs[i] & 1) : 0;
    }
    const int K = ws.st->K;
    for (int k = threadIdx.x; k < K; k += kQThreads) qacc[k] = 0.0;
#pragma unroll
    for (int j = 0; j < kQCells; ++j)
        if (kk[j] < 0 || kk[j] >= K) dd[j] = __builtin_nan("");
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kQCells; ++j)
        if (!isnan(dd[j])) atomicAdd(&qacc[kk[j]], sub_logp(dd[j], sb[j]));
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kQThreads)
        if (qacc[k] != 0.0) atomicAdd(&ws.qsub[k], qacc[k]);
}

void launch_split_ratios(const Ws& ws, const int32_t* c, const uint8_t* cs, int k_guess, hipStream_t s)
{
    if (ws.flags & kFlagSplitQ) {
        const int64_t per = (int64_t)kQThreads * kQCells;
        const int64_t blocks = ws.N > 0 ? (ws.N + per - 1) / per : 1;
        hipLaunchKernelGGL(k_split_q, dim3((unsigned)blocks), dim3(kQThreads), sizeof(double) * (size_t)ws.k_max, s,
                           ws, c, cs);
    }
    launch_sm_pair(ws, 0, k_guess, s);
}

// ---------------------------------------------------------------------------
// Random splits (chain B of Section 2.4).  Each cell draws a fair coin; the
// statistics of the coin halves go to rssub / rnsub through the statistics
// pass (a copy of the workspace view with those arrays in place of ssub /
// nsub), the ratios and decisions run on that view, and the accepted
// clusters' rows and their cells' sub-labels are then committed.
// ---------------------------------------------------------------------------
__global__ void k_rsplit_coins(Ws ws, uint32_t step)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ws.N; i += (int64_t)gridDim.x * blockDim.x)
        ws.rbits[i] = (uint8_t)(philox(ws.seed, (uint32_t)i, 0u, step, kRSplit, 0u).w[0] >> 31);
}

// After the decisions: the split clusters' statistics from the halves (the
// decision kernel has moved half 1 to the new cluster in rssub / rnsub), and
// every cell of a split cluster takes its coin as sub-label, so that the
// relabel sends coin 1 to the new cluster.
__global__ void k_rsplit_apply(Ws ws, const int32_t* __restrict__ c, uint8_t* __restrict__ cs)
{
    const int K0 = ws.st->sm_n;          // clusters before the pass
    const int G = ws.G;
    if (blockIdx.x == 0) {
        for (int k = 0; k < K0; ++k) {
            if (!ws.sm_acc[k]) continue;
            const int j = ws.relab_c[2 * k + 1];
            for (int u = threadIdx.x; u < 2 * G; u += blockDim.x) {
                ws.ssub[(int64_t)2 * k * G + u] = ws.rssub[(int64_t)2 * k * G + u];
                ws.ssub[(int64_t)2 * j * G + u] = ws.rssub[(int64_t)2 * j * G + u];
            }
            if (threadIdx.x < 2) {
                ws.nsub[2 * k + threadIdx.x] = ws.rnsub[2 * k + threadIdx.x];
                ws.nsub[2 * j + threadIdx.x] = ws.rnsub[2 * j + threadIdx.x];
            }
        }
        if (threadIdx.x == 0) {
            ws.st->sm_pass = 2;
            ws.st->rs_live = 0;
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ws.N; i += (int64_t)gridDim.x * blockDim.x) {
        const int k = c[i];
        if (k >= 0 && k < K0 && ws.sm_acc[k]) cs[i] = ws.rbits[i];
    }
}

// With `ready` the coins and the statistics of the halves were built by the
// sub-cluster pass of the sweep before (k_sub_stats) for this step.
void launch_random_split(const Ws& ws, const int32_t* c, uint8_t* cs, uint32_t step, bool ready, int k_guess,
                         hipStream_t s)
{
    int64_t cb = (ws.N + 255) / 256;
    if (cb > 4096) cb = 4096;
    Ws halves = ws;
    halves.ssub = ws.rssub;
    halves.nsub = ws.rnsub;
    if (!ready) {
        hipLaunchKernelGGL(k_rsplit_coins, dim3((unsigned)cb), dim3(256), 0, s, ws, step);
        launch_stats(halves, c, ws.rbits, s);
    }
    launch_sm_pair(halves, 1, k_guess, s);
    launch_sm_decide(halves, 0, step, s);
    hipLaunchKernelGGL(k_rsplit_apply, dim3((unsigned)cb), dim3(256), 0, s, ws, c, cs);
}

void launch_merge_ratios(const Ws& ws, int k_guess, hipStream_t s)
{
    launch_sm_pair(ws, 2, k_guess, s);
    const long long kg = k_grid(ws, k_guess);
    const long long np = kg * (kg - 1) / 2;
    const int mb = np < 4096 ? (int)(np > 0 ? np : 1) : 4096;
    hipLaunchKernelGGL(k_merge_ratios, dim3(mb), dim3(kMergeThreads), 0, s, ws);
}

// ---------------------------------------------------------------------------
// Decisions (one workgroup of 1024 threads).
// ---------------------------------------------------------------------------
constexpr int kDecideThreads = 1024;

__device__ void move_row_pair(Ws& ws, int from, int to)
{
    // statistics and counts of cluster `from` (both sub-clusters) to `to`
    const int G = ws.G;
    for (int u = threadIdx.x; u < 2 * G; u += kDecideThreads)
        ws.ssub[(int64_t)2 * to * G + u] = ws.ssub[(int64_t)2 * from * G + u];
    if (threadIdx.x < 2) ws.nsub[2 * to + threadIdx.x] = ws.nsub[2 * from + threadIdx.x];
    if (threadIdx.x == 0) ws.reset[to] = ws.reset[from];
}

__global__ void __launch_bounds__(kDecideThreads) k_sm_decide(Ws ws, int merge_pass, uint32_t step)
{
    extern __shared__ int32_t lds[];          // 3 k_max ints
    int32_t* newlab = lds;                     // split: new label of sub-cluster 1; merge: target cluster
    int32_t* cmap = lds + ws.k_max;            // compaction map
    int32_t* used = lds + 2 * ws.k_max;        // merge: cluster already merged
    __shared__ unsigned long long rkey[kDecideThreads];
    __shared__ long long ridx[kDecideThreads];
    __shared__ int s_count, s_K, s_any;
    __shared__ int32_t s_wave[kDecideThreads / 64];
    const int t = threadIdx.x;
    // the first candidate of this thread (cluster or pair t) is read and its
    // uniform drawn before K is known (sm_logr has k_max + k_max (k_max - 1) / 2
    // entries)
    const long long nslots = (long long)ws.k_max + (long long)ws.k_max * (ws.k_max - 1) / 2;
    const double lr_t = t < nslots ? ws.sm_logr[t] : __builtin_nan("");
    const Words w_t = philox(ws.seed, (uint32_t)t, 0u, step, merge_pass ? kMerge : kSplit, 0u);
    const double lu_t = log(unit52(w_t.w[0], w_t.w[1]));
    const int K = ws.st->K;
    const int G = ws.G;
    for (int k = t; k < ws.k_max; k += kDecideThreads) {
        newlab[k] = -1;
        used[k] = 0;
    }
    if (t == 0) { s_count = 0; s_any = 0; }
    __syncthreads();

    if (!merge_pass) {
        // acceptance tests in parallel (cluster t is this thread's, K <= k_max
        // <= kDecideThreads), new labels in cluster order
        if (t < K) {
            ws.sm_acc[t] = 0;
            used[t] = isnan(lr_t) ? 0 : (lu_t < lr_t ? 2 : 1);   // 1 proposed, 2 accepted
        }
        __syncthreads();
        // accepted splits take new labels K, K + 1, ... in cluster order while
        // they fit below k_max (workgroup-wide exclusive counts)
        {
            const int ut = t < K ? used[t] : 0;
            int nprop, nacc;
            block_exclusive_count(ut != 0, s_wave, &nprop);
            const int pos = block_exclusive_count(ut == 2, s_wave, &nacc);
            if (ut == 2 && K + pos < ws.k_max) {
                newlab[t] = K + pos;
                ws.sm_acc[t] = 1;
            }
            if (t == 0) {
                const int fit = min(nacc, ws.k_max - K);
                // counters by atomics that return nothing: no round trip before the barrier
                atomicAdd(&ws.st->counters[kCntSplitsProposed], (unsigned long long)nprop);
                atomicAdd(&ws.st->counters[kCntSplitsAccepted], (unsigned long long)fit);
                atomicAdd(&ws.st->counters[kCntKmaxSkips], (unsigned long long)(nacc - fit));
                s_K = K + fit;
                s_any = fit > 0;
            }
        }
        __syncthreads();
        for (int k = 0; k < K; ++k) {
            const int j = newlab[k];
            if (j < 0) continue;
            for (int u = t; u < G; u += kDecideThreads) {
                ws.ssub[(int64_t)(2 * j) * G + u] = ws.ssub[(int64_t)(2 * k + 1) * G + u];
                ws.ssub[(int64_t)(2 * j + 1) * G + u] = 0;
                ws.ssub[(int64_t)(2 * k + 1) * G + u] = 0;
            }
            if (t == 0) {
                ws.nsub[2 * j] = ws.nsub[2 * k + 1];
                ws.nsub[2 * j + 1] = 0;
                ws.nsub[2 * k + 1] = 0;
                ws.reset[k] = 1;
                ws.reset[j] = 1;
            }
            __syncthreads();
        }
        for (int k = t; k < K; k += kDecideThreads) {
            const int j = newlab[k];
            ws.relab_c[2 * k] = k;
            ws.relab_c[2 * k + 1] = j >= 0 ? j : k;
            ws.relab_s[2 * k] = j >= 0 ? 0 : 0xFF;
            ws.relab_s[2 * k + 1] = j >= 0 ? 0 : 0xFF;
        }
        if (t == 0) {
            ws.st->K = s_K;
            if (ws.k_hint) __hip_atomic_store(ws.k_hint, s_K, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            ws.st->relabel = s_any;
            if (s_any) ws.st->relabels += 1;
            ws.st->sm_pass = 0;
            ws.st->sm_n = K;
        }
        return;
    }

    // merge pass: collect the accepted pairs with their random keys
    const long long npairs = (long long)K * (K - 1) / 2;
    for (long long p = t; p < npairs; p += kDecideThreads) {
        ws.sm_acc[p] = 0;
        const bool first = p == t;
        const Words w = first ? w_t : philox(ws.seed, (uint32_t)p, 0u, step, kMerge, 0u);
        const double lu = first ? lu_t : log(unit52(w.w[0], w.w[1]));
        if (lu < (first ? lr_t : ws.sm_logr[p])) {
            const int q = atomicAdd(&s_count, 1);
            ws.mkey[q] = ((unsigned long long)w.w[2] << 32) | w.w[3];
            ws.mlist[q] = (int32_t)p;
        }
    }
    __syncthreads();
    const int ncand = s_count;
    // visit in ascending (key, pair index); a cluster merges at most once
    unsigned long long merges = 0;
    for (;;) {
        unsigned long long bk = ~0ull;
        long long bp = -1;
        for (int q = t; q < ncand; q += kDecideThreads) {
            const long long p = ws.mlist[q];
            int k1, k2;
            pair_of(p, &k1, &k2);
            if (used[k1] || used[k2]) continue;
            const unsigned long long key = ws.mkey[q];
            if (bp < 0 || key < bk || (key == bk && p < bp)) { bk = key; bp = p; }
        }
        rkey[t] = bk;
        ridx[t] = bp;
        __syncthreads();
        for (int off = kDecideThreads / 2; off > 0; off >>= 1) {
            if (t < off) {
                const long long p2 = ridx[t + off];
                if (p2 >= 0 && (ridx[t] < 0 || rkey[t + off] < rkey[t] ||
                                (rkey[t + off] == rkey[t] && p2 < ridx[t]))) {
                    rkey[t] = rkey[t + off];
                    ridx[t] = p2;
                }
            }
            __syncthreads();
        }
        const long long win = ridx[0];
        __syncthreads();
        if (win < 0) break;
        if (t == 0) {
            int k1, k2;
            pair_of(win, &k1, &k2);
            used[k1] = used[k2] = 1;
            newlab[k1] = k1;
            newlab[k2] = k1;
            ws.sm_acc[win] = 1;
        }
        ++merges;
        __syncthreads();
    }
    // apply the merges: the union takes k1's label, its sub-clusters are the
    // two old clusters
    for (int k2 = 0; k2 < K; ++k2) {
        const int k1 = newlab[k2];
        if (k1 < 0 || k1 == k2) continue;
        for (int u = t; u < G; u += kDecideThreads) {
            const unsigned long long a = ws.ssub[(int64_t)(2 * k1) * G + u] + ws.ssub[(int64_t)(2 * k1 + 1) * G + u];
            const unsigned long long b = ws.ssub[(int64_t)(2 * k2) * G + u] + ws.ssub[(int64_t)(2 * k2 + 1) * G + u];
            ws.ssub[(int64_t)(2 * k1) * G + u] = a;
            ws.ssub[(int64_t)(2 * k1 + 1) * G + u] = b;
            ws.ssub[(int64_t)(2 * k2) * G + u] = 0;
            ws.ssub[(int64_t)(2 * k2 + 1) * G + u] = 0;
        }
        if (t == 0) {
            const unsigned long long na = ws.nsub[2 * k1] + ws.nsub[2 * k1 + 1];
            const unsigned long long nb = ws.nsub[2 * k2] + ws.nsub[2 * k2 + 1];
            ws.nsub[2 * k1] = na;
            ws.nsub[2 * k1 + 1] = nb;
            ws.nsub[2 * k2] = ws.nsub[2 * k2 + 1] = 0;
            ws.reset[k1] = 0;
            ws.reset[k2] = 0;
        }
        __syncthreads();
    }
    // compaction of the emptied clusters: the others keep their order
    // (a workgroup-wide exclusive count)
    int nk;
    {
        const bool keep = t < K && !(newlab[t] >= 0 && newlab[t] != t);
        const int pos = block_exclusive_count(keep, s_wave, &nk);
        if (t < K) cmap[t] = keep ? pos : -1;
    }
    if (t == 0) {
        atomicAdd(&ws.st->counters[kCntMergesProposed], (unsigned long long)npairs);
        atomicAdd(&ws.st->counters[kCntMergesAccepted], merges);
    }
    __syncthreads();
    if (merges) {
        for (int k = 0; k < K; ++k) {
            const int j = cmap[k];
            if (j >= 0 && j != k) move_row_pair(ws, k, j);
            __syncthreads();
        }
        for (int k = nk; k < K; ++k) {
            for (int u = t; u < 2 * G; u += kDecideThreads) ws.ssub[(int64_t)2 * k * G + u] = 0;
            if (t < 2) ws.nsub[2 * k + t] = 0;
            if (t == 0) ws.reset[k] = 0;
        }
    }
    for (int k = t; k < K; k += kDecideThreads) {
        const int target = newlab[k] >= 0 ? newlab[k] : k;
        const int lab = cmap[target];
        const uint8_t sub = newlab[k] >= 0 ? (uint8_t)(newlab[k] == k ? 0 : 1) : 0xFF;
        ws.relab_c[2 * k] = lab;
        ws.relab_c[2 * k + 1] = lab;
        ws.relab_s[2 * k] = sub;
        ws.relab_s[2 * k + 1] = sub;
    }
    if (t == 0) {
        ws.st->K = nk;
        if (ws.k_hint) __hip_atomic_store(ws.k_hint, nk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        ws.st->relabel = merges > 0;
        if (merges > 0) ws.st->relabels += 1;
        ws.st->sm_pass = 1;
        ws.st->sm_n = (int32_t)npairs;
    }
}

void launch_sm_decide(const Ws& ws, int merge_pass, uint32_t step, hipStream_t s)
{
    hipLaunchKernelGGL(k_sm_decide, dim3(1), dim3(kDecideThreads), sizeof(int32_t) * 3 * (size_t)ws.k_max, s, ws,
                       merge_pass, step);
}

}  // namespace dpmm
