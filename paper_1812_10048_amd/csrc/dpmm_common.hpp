// dpmm_common.hpp -- definitions shared by the HIP kernels and the host side
// of libdpmm (gfx950).  Nothing here is shared with the CPU oracle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpmm {

// ---------------------------------------------------------------------------
// Random numbers.  Philox4x32-10 (Salmon et al., SC'11) addressed by
// (element, sub-index, step, stream, call): every draw of the sampler has a
// fixed counter, so a chain does not depend on thread scheduling.
// ---------------------------------------------------------------------------
enum Stream : uint32_t {
    kInit = 1,      // initial labels
    kGamma = 2,     // Gamma variates of theta and thetabar
    kPi = 3,        // Gamma variates of the mixing proportions
    kGumbelC = 4,   // Gumbel noise of the cluster choice
    kGumbelS = 5,   // Gumbel noise of the sub-cluster choice
    kResub = 6,     // fair coins of a reset cluster's sub-labels
    kChain = 7,     // split chain or merge chain
    kSplit = 8,     // split acceptance
    kMerge = 9,     // merge acceptance and visiting order
    kRSplit = 10    // per-cell coins of a random split
};

constexpr uint32_t kSubRowBase = 0x10000u;   // Philox row id of thetabar_{k,r} = base + 2k + r
constexpr uint32_t kAlphaElement = 0xFFFFFFFFu;
constexpr int kGammaTries = 64;

struct Words { uint32_t w[4]; };

__host__ __device__ inline Words philox(uint64_t seed, uint32_t element, uint32_t sub, uint32_t step,
                                        uint32_t stream, uint32_t call)
{
    uint32_t x0 = element, x1 = sub, x2 = step, x3 = (stream << 24) | (call & 0xFFFFFFu);
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product gives both halves (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0, p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Words o;
    o.w[0] = x0; o.w[1] = x1; o.w[2] = x2; o.w[3] = x3;
    return o;
}

// (w >> 9 + 1/2) 2^-23: an odd multiple of 2^-24, exact in float and double.
__host__ __device__ inline float unit23f(uint32_t w) { return ((float)(w >> 9) + 0.5f) * 0x1p-23f; }
__host__ __device__ inline double unit23d(uint32_t w) { return ((double)(w >> 9) + 0.5) * 0x1p-23; }
// 52 random bits from two words, an odd multiple of 2^-53, exact in double.
__host__ __device__ inline double unit52(uint32_t hi, uint32_t lo)
{
    return ((double)((((uint64_t)hi << 32) | lo) >> 12) + 0.5) * 0x1p-52;
}

// ---------------------------------------------------------------------------
// Device-resident scalars of a context (K changes on the device).
// ---------------------------------------------------------------------------
enum Counter {
    kCntGammaCaps = 0,
    kCntSplitsProposed = 1,
    kCntSplitsAccepted = 2,
    kCntMergesProposed = 3,
    kCntMergesAccepted = 4,
    kCntKmaxSkips = 5,
    kCntRefined = 6,
    kCntEvals = 7,        // sum over sweeps of N (K + 2)
    kCntNearTie = 8,      // cluster decisions whose FP64 relative margin is below kNearTie
    kNumCounters = 9
};

// Relative Gumbel-max margin (top1 - top2) / max(1, |top1|) below which a
// decision is a near tie: counted, and always taken in FP64.
constexpr double kNearTie = 1e-6;

// optional per-cell score dump of a sweep, FP32 or FP64
__host__ __device__ inline void put_dbg(void* dbg, int dbg64, int64_t idx, double v)
{
    if (dbg64) reinterpret_cast<double*>(dbg)[idx] = v;
    else reinterpret_cast<float*>(dbg)[idx] = (float)v;
}

struct DevState {
    int32_t K;            // current number of clusters
    int32_t relabel;      // nonzero if the relabel map must be applied to the labels
    int32_t sm_pass;      // 0 split, 1 merge (last split/merge call)
    int32_t sm_n;         // candidates of the last split/merge call
    int32_t n_refine;     // cells queued for FP64 re-scoring in the current sweep
    int32_t data_error;   // CSR validation failures
    int32_t has_new;      // 1 while cluster K - 1 is the new cluster of the current sweep
    int32_t pad;
    unsigned long long counters[kNumCounters];
    double log_joint;     // written by launch_log_joint
    uint32_t relabels;    // times the labels were renumbered (compaction, accepted moves)
    int32_t lay_go;       // the cluster-sorted copy is being rebuilt (gate of its kernels)
    int32_t lay_nblk;     // blocks of the copy
    int32_t lay_K;        // K when the copy was built
    uint32_t lay_relabels;   // relabels when the copy was built
    int32_t rs_live;      // the coin-half statistics of the next random split are in rssub / rnsub
    int32_t n_mov;        // cells queued for the packed-matrix sub-cluster draw (split-BF16 sweeps)
    int32_t pad3;
};

// Packed count entry: gene in the low 16 bits, count in the high 16 bits.
// Rows are padded to a multiple of 4 entries (16 bytes) with kPadEntry.
constexpr uint32_t kPadEntry = 0x0000FFFFu;   // gene 0xFFFF, count 0

constexpr int kBlkCells = 256;
constexpr int kLayDmax = 8;                        // dense gene chunks per block of the cluster-sorted copy
constexpr int kDenseChunkBytes = 256 * 64;         // one byte per (cell, gene) of a block and chunk
constexpr uint32_t kFlagSplitQ = 1u;          // dpmm_params.flags bit of the split proposal term
constexpr uint32_t kFlagNewCluster = 2u;      // ... and of the Gibbs step over K + 1 clusters
constexpr uint32_t kFlagRandomSplit = 4u;     // ... and of the random-split pass
constexpr int kBlkGenes = 64;
// cost of a tail entry against a dense byte in the choice of a block's dense
// chunks (layout.hip): its 4 bytes, the gather of its gene's FP32 row of log
// theta, and its place in the serial tail walk, where a wavefront waits for
// its longest tail (measured: 72-192 equally fast at 1.3M x 2000, 36 slower)
constexpr long long kTailCost = 96;
constexpr int kPlaneGenes = 32;                    // places of chunk 0 that the high plane covers (one k-step)
constexpr int kMaxClusters = 1024;                 // largest k_max dpmm_init accepts
constexpr int kSubDigits = 7;                      // digit columns after the K clusters in lay_bhi (layout.hip)
constexpr int kSpanBlocks = 128;                   // blocks per span of the statistics reduction (laysub.hip)
// spans of the reduction: each cluster's blocks are cut separately
__host__ __device__ inline int32_t lay_spans(int32_t nblk_cap, int32_t k_max) { return nblk_cap / kSpanBlocks + k_max; }

// Refine-queue flags (high bits of a queued cell index).
constexpr uint32_t kRefineCluster = 1u << 31;
constexpr uint32_t kRefineSub = 1u << 30;
constexpr uint32_t kRefineMask = (1u << 30) - 1;

#if defined(__HIPCC__)
// Exclusive count of `on` over the threads below this one, and the total, for
// a workgroup of whole wavefronts (one flag per thread): ballots per
// wavefront, then the wavefront totals through LDS (s_wave: blockDim.x / 64
// words).  Every thread of the workgroup must call it.
__device__ inline int block_exclusive_count(bool on, int32_t* s_wave, int* total)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const unsigned long long m = __ballot(on);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[w] = __popcll(m);
    __syncthreads();
    int base = 0, tot = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
        const int c = s_wave[q];
        if (q < w) base += c;
        tot += c;
    }
    __syncthreads();                   // (s_wave may be reused)
    *total = tot;
    return base + below;
}

#endif

// Row walker: entries are read 16 bytes at a time (rows start and end on
// 16-byte boundaries) with the next block already in flight.
#if defined(__HIPCC__)
// Entries [q, q + 4) of a row ending at e, or four padding entries when
// q >= e.  The load is unconditional, from q clamped to the row start b (the
// entry array has 16 bytes of slack past its end), and the padding is chosen
// as a value: a select between a load and a local would turn into a select of
// addresses that puts the local in private memory.
__device__ inline uint4 load_entries(const uint32_t* ent, int64_t q, int64_t b, int64_t e)
{
    const uint4 v = *reinterpret_cast<const uint4*>(ent + (q < e ? q : b));
    return q < e ? v : make_uint4(kPadEntry, kPadEntry, kPadEntry, kPadEntry);
}

struct RowCursor {
    int64_t pos, beg, end;
    uint4 cur, nxt;
    __device__ inline void start(const uint32_t* ent, int64_t b, int64_t e)
    {
        pos = b;
        beg = b;
        end = e;
        cur = load_entries(ent, b, b, e);
        nxt = load_entries(ent, b + 4, b, e);
    }
    __device__ inline uint32_t peek() const
    {
        const int sl = (int)(pos & 3);
        return sl == 0 ? cur.x : sl == 1 ? cur.y : sl == 2 ? cur.z : cur.w;
    }
    __device__ inline void advance(const uint32_t* ent)
    {
        ++pos;
        if ((pos & 3) == 0) {
            cur = nxt;
            nxt = load_entries(ent, pos + 4, beg, end);
        }
    }
};
#endif

#if defined(__HIPCC__)
// The sub-cluster draw of eq. 8 for a cell of cluster k, shared by the passes
// over the packed matrix and over the cluster-sorted copy.  Weights: nbar_{k,r}
// at the start of the sweep, less one for the sub-cluster the cell was in
// (code: 1 + its old sub-label if it was in k, else 0).
struct SubWeights {
    double l0, l0m, l1, l1m;
};
__device__ inline double log_count(long long w) { return w > 0 ? log((double)w) : -INFINITY; }
__device__ inline SubWeights sub_weights(const unsigned long long* nsub_prev, int k)
{
    const long long n0 = (long long)nsub_prev[2 * k], n1 = (long long)nsub_prev[2 * k + 1];
    return SubWeights{log_count(n0), log_count(n0 - 1), log_count(n1), log_count(n1 - 1)};
}
// FP32 Gumbel noise of sub-cluster 1 less that of sub-cluster 0
__device__ inline float sub_noise(uint64_t seed, uint32_t i, uint32_t step, uint32_t stream)
{
    const Words w = philox(seed, i, 0u, step, stream, 0u);
    return (-logf(-logf(unit23f(w.w[1])))) - (-logf(-logf(unit23f(w.w[0]))));
}
// The draw given df = sum_u x_u (log thetabar_{k,1,u} - log thetabar_{k,0,u})
// in FP64; dd (the FP64 score difference with the weights) is returned for
// the split proposal term.  The draw compares dd + g1 - g0 with 0: the FP32
// noise is within 3e-6 of the FP64 noise, so when the FP32 difference clears
// tau its sign is the FP64 sign; otherwise (or with a zero weight) the FP64
// comparison decides.
__device__ inline int sub_draw(uint64_t seed, uint32_t i, uint32_t step, uint32_t stream, const SubWeights& w,
                               int code, float nd, double df, double* dd_out)
{
    double lw0 = code == 1 ? w.l0m : w.l0;
    double lw1 = code == 2 ? w.l1m : w.l1;
    if (!(lw0 > -INFINITY) && !(lw1 > -INFINITY)) lw0 = lw1 = 0.0;   // both weights zero: equal
    const double dd = lw1 - lw0 + df;
    *dd_out = dd;
    const float d32 = (float)dd + nd;
    const float tau = 1e-3f + 1e-5f * fabsf((float)dd);
    if (isfinite(dd) && fabsf(d32) > tau) return d32 > 0.0f ? 1 : 0;
    const Words wd = philox(seed, i, 0u, step, stream, 0u);
    const double v0 = lw0 + (-log(-log(unit23d(wd.w[0]))));
    const double v1 = lw1 + df + (-log(-log(unit23d(wd.w[1]))));
    return v1 > v0 ? 1 : 0;
}
// log p(cbar_i) of eq. 8 for the split proposal term: a two-way softmax of
// the scores, whose difference is dd
__device__ inline double sub_logp(double dd, int sub)
{
    const double x = sub ? -dd : dd;
    return -(fmax(x, 0.0) + log1p(exp(-fabs(x))));
}
#endif

// Top bits of srow.w after a sort by new cluster: 1 + the cell's sub-label
// before the sweep if it was already in that cluster, else 0.
constexpr int kSrowOldShift = 30;
constexpr uint32_t kSrowLenMask = (1u << kSrowOldShift) - 1u;

// Genes per workgroup of the parameter redraw, and the tiles of a row.
constexpr int kRedrawGenes = 256;
__host__ __device__ inline int redraw_tiles(int G) { return (G + kRedrawGenes - 1) / kRedrawGenes; }

// Genes per workgroup of the split-ratio and cluster-logDM passes, the tiles of
// a cluster, and one tile's partial result (compensated sum s + c of the
// per-gene terms, sum of beta_u, and the count sums of the two halves).
constexpr int kSmGenes = 512;
// Counts below kRiseTab take lgamma(beta_u + v) - lgamma(beta_u) from a
// per-gene table (refreshed with lgbeta) instead of the recurrence.
constexpr int kRiseTab = 16;
__host__ __device__ inline int sm_tiles(int G) { return (G + kSmGenes - 1) / kSmGenes; }
struct SmPart {
    double s, c, beta;
    long long a, b;
};

// ---------------------------------------------------------------------------
// View of the workspace, passed by value to kernels.
// ---------------------------------------------------------------------------
struct Ws {
    int64_t N;
    int32_t G;
    int32_t k_max;
    int32_t Gpad;          // nch x kBlkGenes: G rounded up to an even number of gene chunks
    int32_t kpad;          // k_max rounded up to a multiple of 16
    double alpha;
    uint64_t seed;

    const uint32_t* ent;   // [nnz_pad] packed entries
    const int64_t* roff;   // [N + 1] padded row offsets (multiples of 4)
    DevState* st;
    uint8_t* reset;        // [k_max]
    unsigned long long* nsub;   // [2 k_max]
    unsigned long long* ssub;   // [2 k_max G]   (k, r, u) at (2k + r) G + u
    double* beta;          // [G]
    double* lgbeta;        // [G] lgamma(beta_u), refreshed wherever beta is written (init, set_beta, EB update)
    double* lgrise;        // [G][kRiseTab] lgamma(beta_u + v) - lgamma(beta_u), 0 at v = 0; refreshed with lgbeta
    double* logpi;         // [k_max]
    double* lt64;          // [3 k_max G]: rows k, then k_max + 2k + r
    float* lc32;           // [G][kpad] cluster log theta, gene-major
    float2* ls32;          // [G][k_max] sub-cluster log theta pairs, gene-major
    uint16_t* lhi;         // split-BF16 tables, see assign_mfma.hip
    uint16_t* llo;
    uint32_t* refine;      // [N] queued cells with flags
    int32_t* perm;         // [N] cells sorted by group 2k + r (processing order of a sweep)
    uint4* srow;           // [N] per sorted position: (cell, row offset lo, hi, row length | old << kSrowOldShift)
    int32_t* grp_cnt;      // [2 k_max] group sizes
    int32_t* grp_off;      // [2 k_max + 1] group offsets in perm
    int32_t* grp_cur;      // [2 k_max] scatter cursors
    unsigned long long* nsub_prev;   // [2 k_max] n_{k,r} at the start of the sweep
    // cluster-sorted copy of the counts for the matrix cores (split-BF16,
    // layout.hip): blocks of kBlkCells cells of one cluster, genes renumbered
    // per cluster, the first D_b chunks of kBlkGenes genes dense (one byte per
    // count, MFMA fragment order), the other entries in per-cell tail lists
    int32_t* lay_kc;       // [nblk_cap] layout cluster of each block
    int32_t* lay_pbeg;     // [nblk_cap] its first cell in the sort order
    int32_t* lay_pcnt;     // [nblk_cap] its number of cells
    int32_t* lay_cell;     // [nblk_cap kBlkCells] cell of each slot, -1 if empty
    int64_t* lay_doff;     // [nblk_cap + 1] dense chunks before each block
    int64_t* lay_toff;     // [nblk_cap kBlkCells + 1] tail entries before each slot
    uint8_t* lay_dense;    // dense chunks, kDenseChunkBytes each
    uint32_t* lay_tail;    // tail entries (gene | count << 16), each slot's in row order
    uint16_t* lay_nnz;     // [nblk_cap kBlkCells] the products of each slot's cell that its scores sum
                           // (its non-zero counts, plus one for each count split by the high plane)
    uint8_t* lay_hcnt;     // [nblk_cap kBlkCells] the slot's high-plane entries, last in its tail
    uint8_t* lay_bh;       // [nblk_cap] 1 when the block has a high plane (one more chunk after its D)
    uint16_t* lay_rank;    // [k_max G] place of gene u in cluster L's order
    uint16_t* lay_gene;    // [k_max kLayDmax kBlkGenes] gene at place j
    uint16_t* lay_bhi;     // [k_max][lay_cols][kLayDmax kBlkGenes] hi of log theta in L's gene order
    uint16_t* lay_blo;     // same for lo
    uint64_t* lay_lim;     // [k_max][kLayDmax][2][8][4] base-256 digits of the fixed-point delta (laysub.hip)
    int32_t* lay_dE;       // [k_max] its binary scale
    int32_t* lay_dS;       // [k_max][kLayDmax + 1][8] digit sums over the first D chunks
    double* lay_dfull;     // [k_max][G] the difference itself, gene-major (tail entries)
    double* lay_sw;        // [k_max][4] the sub-cluster weights of the draw (SubWeights)
    uint32_t* lay_part;    // [nblk_cap][lay_pw] a block's count sums per (sub-cluster | coin, place of its cluster)
    int32_t lay_pw;        // rows x kLayDmax kBlkGenes words of those histograms (rows 4 with random splits, else 2)
    int32_t* lay_bbeg;     // [k_max + 1] first block of each layout cluster
    int32_t* lay_sbeg;     // [k_max + 1] spans (of up to 32 blocks) before each layout cluster's first
    uint32_t* mov;         // [N] cells of a block whose new cluster is not the block's (laysub.hip)
    int32_t nblk_cap;      // blocks the copy can hold: ceil(N / kBlkCells) + k_max
    int32_t lay_cols;      // column rows per layout cluster in lay_bhi / lay_blo
    int32_t sub_cells;     // sorted cells per workgroup of the sub-cluster/statistics pass
    uint32_t flags;        // kFlagSplitQ: the split ratio carries -sum log p(cbar_i)
    double* subdd;         // [N] the score difference dd of the cell's draw of eq. 8 in the last sweep, NaN
                           // for a cell of a reset cluster (with kFlagSplitQ only; log p(cbar_i) = sub_logp)
    double* qsub;          // [k_max] sum of log p(cbar_i) over the cells of each cluster (split pass)
    uint8_t* rbits;        // [N] coins of the last random-split pass (with kFlagRandomSplit)
    unsigned long long* rssub;   // [2 k_max G] statistics of the coin halves
    unsigned long long* rnsub;   // [2 k_max] sizes of the coin halves
    int32_t* k_hint;       // mapped pinned host word: K after the last compaction or split/merge
                           // (a launch-size hint for the host; written by the kernels that set K)
    int32_t* relab_c;      // [2 k_max] new cluster of an old (k, r)
    uint8_t* relab_s;      // [2 k_max] new sub-label of an old (k, r); 0xFF keeps it
    double* sm_logr;       // [k_max + k_max (k_max - 1) / 2]
    uint8_t* sm_acc;       // same size
    unsigned long long* mkey;   // same size: random keys of accepted merge pairs
    int32_t* mlist;        // same size: their pair indices
    double* dm_k;          // [k_max] logDM of each cluster's statistics
    double* eb_tmp;        // [k_max + G] scratch of the empirical-Bayes step
    double2* rd_part;      // [3 k_max + 1][redraw_tiles(G)] (max, sum exp) of each gene tile of a redrawn row
    SmPart* sm_part;       // [k_max][sm_tiles(G)] partial results of the split-ratio / logDM passes
};

}  // namespace dpmm
