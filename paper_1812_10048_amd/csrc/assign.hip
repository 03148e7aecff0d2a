// assign.hip -- steps a2-a3 on the vector ALUs: per-cell log-likelihoods
// S_ik = sum_u x_i^u log theta_{k,u} (eq. 26) against every cluster and the
// Gumbel-max draw of c_i (eq. 4, third line).
//
// Layout: one thread per cell, 256 cells per workgroup.  log theta is staged
// through LDS one chunk of kChunk genes at a time ([gene][cluster], so one
// entry reads KT consecutive values); each thread walks its own packed row
// in step with the chunks, so a row is read once per cluster group.
//
// In FP32 every cluster decision carries a certified rounding bound: the sum
// of n same-sign products in FP32 is within (n + 4) 2^-24 |sum| of the exact
// sum over the FP64 parameters (all terms x log theta are <= 0), and the FP32
// Gumbel noise is within 1e-5.  A decision whose Gumbel gap is inside the
// bound is queued for the FP64 re-score (k_refine), so the final labels are
// the FP64 decisions.  The sub-cluster draw follows in k_sub_stats.  Cells
// are taken in the order of the last sort (cells of a cluster together).
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

constexpr int kAssignThreads = 256;
constexpr int kChunk = 128;

template <typename T> __device__ inline T gumbel_of(uint32_t w);
template <> __device__ inline float gumbel_of<float>(uint32_t w) { return -logf(-logf(unit23f(w))); }
template <> __device__ inline double gumbel_of<double>(uint32_t w) { return -log(-log(unit23d(w))); }

template <typename T> __device__ inline T log_of(T v);
template <> __device__ inline float log_of<float>(float v) { return logf(v); }
template <> __device__ inline double log_of<double>(double v) { return log(v); }

// rounding bound of an FP32 score built from n products, |acc| and |lp|
__device__ inline float score_bound(float acc, float lp, int64_t n)
{
    return (float)(n + 4) * 0x1p-24f * (fabsf(acc) + fabsf(lp) + 20.0f) + 1e-5f;
}

__device__ inline float rel_margin(float top1, float top2)
{
    return (top1 - top2) / fmaxf(1.0f, fabsf(top1));
}

// LDS row strides: padded so that consecutive gene rows start on different
// bank groups (rows of 64 floats would all start on bank 0).
template <typename T, int KT> struct Stride { static constexpr int v = KT + (sizeof(T) == 4 ? 4 : 2); };
constexpr int kTabBytes = 34816;    // 128 x 68 x 4 = 128 x 34 x 8

// Stage the [kChunk genes][KT clusters] slice of log theta into LDS.
template <typename T, int KT>
__device__ inline void stage_chunk(const Ws& ws, T* tab, int c0, int kb, int K)
{
    constexpr int S = Stride<T, KT>::v;
    for (int idx = threadIdx.x; idx < kChunk * KT; idx += kAssignThreads) {
        int g, k;
        if (sizeof(T) == 4) { g = idx / KT; k = idx % KT; }          // FP32 table is [G][kpad]
        else { k = idx / kChunk; g = idx % kChunk; }                 // FP64 table is [k][G]
        const int gg = c0 + g, kk = kb + k;
        T v = 0;
        if (gg < ws.G && kk < K) {
            if (sizeof(T) == 4) v = (T)ws.lc32[(int64_t)gg * ws.kpad + kk];
            else v = (T)ws.lt64[(int64_t)kk * ws.G + gg];
        }
        tab[g * S + k] = v;
    }
}

template <typename T>
struct Top2 {
    T v1, v2;     // best and second-best Gumbel-perturbed scores
    T a1, a2;     // their log-likelihoods
    T p1, p2;     // their log pi
    int k1;
};

template <typename T, int KT>
__device__ void cluster_pass(const Ws& ws, const AssignArgs& a, T* tab, int64_t i, bool valid, int64_t b,
                             int64_t e, int K, Top2<T>& top)
{
    constexpr int S = Stride<T, KT>::v;
    for (int kb = 0; kb < K; kb += KT) {
        T acc[KT];
#pragma unroll
        for (int k = 0; k < KT; ++k) acc[k] = 0;
        RowCursor rc;
        rc.start(ws.ent, b, e);
        for (int c0 = 0; c0 < ws.G; c0 += kChunk) {
            __syncthreads();
            stage_chunk<T, KT>(ws, tab, c0, kb, K);
            __syncthreads();
            while (rc.pos < e) {
                const uint32_t en = rc.peek();
                const int g = (int)(en & 0xFFFFu);
                if (g >= c0 + kChunk) break;
                const T x = (T)(en >> 16);
                const T* trow = tab + (g - c0) * S;
#pragma unroll
                for (int k = 0; k < KT; ++k) acc[k] = fma(x, trow[k], acc[k]);
                rc.advance(ws.ent);
            }
        }
        if (!valid) continue;
        // fully unrolled with guards (no early exit), four clusters per Philox
        // call: every index into acc and the words is a constant, so both
        // stay in registers
#pragma unroll
        for (int k4 = 0; k4 < KT; k4 += 4) {
            if (kb + k4 >= K) continue;
            const Words w = philox(ws.seed, (uint32_t)i, (uint32_t)((kb + k4) >> 2), a.step, kGumbelC, 0u);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int kk = kb + k4 + q;
                if (kk >= K) continue;
                const T lp = (T)ws.logpi[kk];
                const T v = lp + acc[k4 + q] + gumbel_of<T>(w.w[q]);
                if (a.dbg && K + 2 <= a.dbg_stride) put_dbg(a.dbg, a.dbg64, i * a.dbg_stride + kk, (double)acc[k4 + q]);
                if (v > top.v1) {
                    top.v2 = top.v1; top.a2 = top.a1; top.p2 = top.p1;
                    top.v1 = v; top.a1 = acc[k4 + q]; top.p1 = lp; top.k1 = kk;
                } else if (v > top.v2) {
                    top.v2 = v; top.a2 = acc[k4 + q]; top.p2 = lp;
                }
            }
        }
    }
}

template <typename T, int KT>
__global__ void __launch_bounds__(kAssignThreads) k_assign_valu(Ws ws, AssignArgs a)
{
    __shared__ __attribute__((aligned(16))) T tab[kTabBytes / sizeof(T)];
    const int K = ws.st->K;
    // cells in the order of the last statistics pass (grouped by cluster)
    const int64_t slot = (int64_t)blockIdx.x * kAssignThreads + threadIdx.x;
    const bool valid = slot < ws.N;
    const int64_t i = valid ? (int64_t)ws.perm[slot] : 0;
    const int64_t b = valid ? ws.roff[i] : 0;
    const int64_t e = valid ? ws.roff[i + 1] : 0;

    Top2<T> top;
    top.v1 = top.v2 = -INFINITY;
    top.a1 = top.a2 = top.p1 = top.p2 = 0;
    top.k1 = 0;
    cluster_pass<T, KT>(ws, a, tab, i, valid, b, e, K, top);

    uint32_t flags = 0;
    if (valid && sizeof(T) == 4 && a.refine && K >= 2) {
        const float gap = (float)(top.v1 - top.v2);
        const float bnd = score_bound((float)top.a1, (float)top.p1, e - b) +
                          score_bound((float)top.a2, (float)top.p2, e - b);
        // within the bound plus the near-tie margin: the FP64 decision could
        // differ, or be a near tie (counted by the re-score)
        const float near = (float)kNearTie * fmaxf(1.0f, fabsf((float)top.v1));
        if (gap <= bnd + near || rel_margin((float)top.v1, (float)top.v2) < a.refine_tol) flags |= kRefineCluster;
    }
    if (valid && sizeof(T) == 8 && K >= 2 &&
        (double)(top.v1 - top.v2) / fmax(1.0, fabs((double)top.v1)) < kNearTie)
        atomicAdd(&ws.st->counters[kCntNearTie], 1ull);

    if (!valid) return;
    const int k = top.k1;
    a.c_new[i] = k;
    if (flags) {
        const int q = atomicAdd(&ws.st->n_refine, 1);
        if (q < ws.N) ws.refine[q] = (uint32_t)i | flags;
    }
}

// The cluster-group width KT is fixed at launch while K lives on the device:
// the host passes the last K it has seen (k_hint); a larger K is covered by
// the kernel's loop over groups of KT clusters.
template <typename T, int KT>
static void launch_kt(const Ws& ws, const AssignArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((k_assign_valu<T, KT>), dim3((unsigned)((ws.N + kAssignThreads - 1) / kAssignThreads)),
                       dim3(kAssignThreads), 0, s, ws, a);
}

void launch_assign_fp32(const Ws& ws, const AssignArgs& a, hipStream_t s)
{
    const int k = a.k_hint > 0 ? a.k_hint : ws.k_max;
    if (k <= 16) launch_kt<float, 16>(ws, a, s);
    else if (k <= 32) launch_kt<float, 32>(ws, a, s);
    else if (k <= 48) launch_kt<float, 48>(ws, a, s);
    else launch_kt<float, 64>(ws, a, s);
}

void launch_assign_fp64(const Ws& ws, const AssignArgs& a, hipStream_t s)
{
    const int k = a.k_hint > 0 ? a.k_hint : ws.k_max;
    if (k <= 16) launch_kt<double, 16>(ws, a, s);
    else launch_kt<double, 32>(ws, a, s);
}

// ---------------------------------------------------------------------------
// FP64 re-score of queued cluster decisions: all K scores with FP64
// log theta gathered from the FP64 table and FP64 Gumbel noise.
// ---------------------------------------------------------------------------
__device__ inline double row_dot64(const Ws& ws, int64_t b, int64_t e, const double* lrow)
{
    double s = 0.0;
    for (int64_t pos = b; pos < e; ++pos) {
        const uint32_t en = ws.ent[pos];
        const uint32_t x = en >> 16;
        if (x) s = fma((double)x, lrow[en & 0xFFFFu], s);
    }
    return s;
}

__global__ void k_refine(Ws ws, AssignArgs a)
{
    const int n = min(ws.st->n_refine, (int)min((int64_t)0x7FFFFFFF, ws.N));
    const int K = ws.st->K;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const uint32_t item = ws.refine[q];
        const int64_t i = (int64_t)(item & kRefineMask);
        if (i >= ws.N) continue;
        const int64_t b = ws.roff[i], e = ws.roff[i + 1];
        int k = a.c_new[i];
        if (item & kRefineCluster) {
            double best = -INFINITY, second = -INFINITY;
            int bk = 0;
            Words w{};
            for (int kk = 0; kk < K; ++kk) {
                if ((kk & 3) == 0) w = philox(ws.seed, (uint32_t)i, (uint32_t)(kk >> 2), a.step, kGumbelC, 0u);
                const double v = ws.logpi[kk] + row_dot64(ws, b, e, ws.lt64 + (int64_t)kk * ws.G) +
                                 gumbel_of<double>(w.w[kk & 3]);
                if (v > best) { second = best; best = v; bk = kk; }
                else if (v > second) second = v;
            }
            k = bk;
            if (K >= 2 && (best - second) / fmax(1.0, fabs(best)) < kNearTie)
                atomicAdd(&ws.st->counters[kCntNearTie], 1ull);
        }
        a.c_new[i] = k;
        atomicAdd(&ws.st->counters[kCntRefined], 1ull);
    }
}

// ---------------------------------------------------------------------------
// FP64 scores of listed cells (debug output): one workgroup per listed cell,
// one thread per column, each walking the cell's packed row.
// ---------------------------------------------------------------------------
__global__ void k_dump_scores(Ws ws, const int32_t* c, const int32_t* cells, int32_t m, double* out)
{
    const int K = ws.st->K;
    for (int j = blockIdx.x; j < m; j += gridDim.x) {
        const int64_t i = cells[j];
        if (i < 0 || i >= ws.N) continue;
        const int64_t b = ws.roff[i], e = ws.roff[i + 1];
        const int k = c[i];
        for (int col = threadIdx.x; col < K + 2; col += blockDim.x) {
            const int row = col < K ? col : ws.k_max + 2 * k + (col - K);
            out[(int64_t)j * (K + 2) + col] = row_dot64(ws, b, e, ws.lt64 + (int64_t)row * ws.G);
        }
    }
}

void launch_dump_scores(const Ws& ws, const int32_t* c, const int32_t* cells, int32_t m, double* out, hipStream_t s)
{
    const int blocks = m < 4096 ? (m > 0 ? m : 1) : 4096;
    hipLaunchKernelGGL(k_dump_scores, dim3(blocks), dim3(64), 0, s, ws, c, cells, m, out);
}

void launch_refine(const Ws& ws, const AssignArgs& a, hipStream_t s)
{
    int64_t blocks = (ws.N + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_refine, dim3((unsigned)blocks), dim3(256), 0, s, ws, a);
}

}  // namespace dpmm
