// assign.hip -- steps a2-a3 on the vector ALUs: per-cell log-likelihoods
// S_ik = sum_u x_i^u log theta_{k,u} (eq. 26) against every cluster, the
// Gumbel-max draw of c_i (eq. 4, third line), then the two sub-cluster
// log-likelihoods of the chosen cluster and the draw of cbar_i (eq. 8).
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
// the FP64 decisions.  The sub-cluster scores (two per cell) are FP64.
// Cells are taken in the order of the last statistics pass, which groups the
// cells of a cluster together.
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
constexpr int kSubChunkF = 64;      // genes per sub-cluster chunk, FP32
constexpr int kSubChunkD = 32;      // genes per sub-cluster chunk, FP64
constexpr int kSubMaxK = 64;        // sub-cluster tables staged in LDS up to this K
constexpr int kTabBytes = 34816;    // max(128 x 68 x 4, 64 x 132 x 4, 128 x 34 x 8, 32 x 130 x 8)

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

// Row walker: entries are read 16 bytes at a time (rows start and end on
// 16-byte boundaries) with the next block already in flight.
struct RowCursor {
    int64_t pos, end;
    uint4 cur, nxt;
    __device__ inline void start(const uint32_t* ent, int64_t b, int64_t e)
    {
        pos = b;
        end = e;
        const uint4 pad = make_uint4(kPadEntry, kPadEntry, kPadEntry, kPadEntry);
        cur = b < e ? *reinterpret_cast<const uint4*>(ent + b) : pad;
        nxt = b + 4 < e ? *reinterpret_cast<const uint4*>(ent + b + 4) : pad;
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
            nxt = pos + 4 < end ? *reinterpret_cast<const uint4*>(ent + pos + 4)
                                : make_uint4(kPadEntry, kPadEntry, kPadEntry, kPadEntry);
        }
    }
};

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
        Words w{};
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            const int kk = kb + k;
            if (kk >= K) break;
            if ((k & 3) == 0) w = philox(ws.seed, (uint32_t)i, (uint32_t)(kk >> 2), a.step, kGumbelC, 0u);
            const T lp = (T)ws.logpi[kk];
            const T v = lp + acc[k] + gumbel_of<T>(w.w[k & 3]);
            if (a.dbg && K + 2 <= a.dbg_stride) a.dbg[i * a.dbg_stride + kk] = (float)acc[k];
            if (v > top.v1) {
                top.v2 = top.v1; top.a2 = top.a1; top.p2 = top.p1;
                top.v1 = v; top.a1 = acc[k]; top.p1 = lp; top.k1 = kk;
            } else if (v > top.v2) {
                top.v2 = v; top.a2 = acc[k]; top.p2 = lp;
            }
        }
    }
}

// Log-likelihoods of the two sub-clusters of cluster k (eq. 8).  For K up to
// kSubMaxK the [genes][K x 2] sub-cluster table is staged through LDS chunk by
// chunk (every thread takes part in the staging, `need` says whether this
// thread's cell uses it); beyond that the values are gathered from memory.
template <typename T>
__device__ void sub_pass(const Ws& ws, T* tab, int64_t b, int64_t e, int K, int k, bool need, T& s0, T& s1)
{
    s0 = 0;
    s1 = 0;
    if (K <= kSubMaxK) {
        constexpr int SC = sizeof(T) == 4 ? kSubChunkF : kSubChunkD;
        const int w2 = 2 * K;
        const int S2 = w2 + (sizeof(T) == 4 ? 4 : 2);
        RowCursor rc;
        rc.start(ws.ent, b, need ? e : b);
        for (int c0 = 0; c0 < ws.G; c0 += SC) {
            __syncthreads();
            for (int idx = threadIdx.x; idx < SC * w2; idx += kAssignThreads) {
                int g, q;
                if (sizeof(T) == 4) { g = idx / w2; q = idx % w2; }   // [G][k_max] pairs, contiguous in q
                else { q = idx / SC; g = idx % SC; }                  // rows k_max + q of the FP64 table
                const int gg = c0 + g;
                T v = 0;
                if (gg < ws.G) {
                    if (sizeof(T) == 4) v = (T)reinterpret_cast<const float*>(ws.ls32)[((int64_t)gg * ws.k_max) * 2 + q];
                    else v = (T)ws.lt64[(int64_t)(ws.k_max + q) * ws.G + gg];
                }
                tab[g * S2 + q] = v;
            }
            __syncthreads();
            if (!need) continue;
            while (rc.pos < rc.end) {
                const uint32_t en = rc.peek();
                const int g = (int)(en & 0xFFFFu);
                if (g >= c0 + SC) break;
                const T x = (T)(en >> 16);
                const T* p = tab + (g - c0) * S2 + 2 * k;
                s0 = fma(x, p[0], s0);
                s1 = fma(x, p[1], s1);
                rc.advance(ws.ent);
            }
        }
        return;
    }
    if (!need) return;
    if (sizeof(T) == 4) {
        const float2* ls = ws.ls32;
        for (int64_t pos = b; pos < e; ++pos) {
            const uint32_t en = ws.ent[pos];
            const T x = (T)(en >> 16);
            if (x == 0) continue;
            const float2 p = ls[(int64_t)(en & 0xFFFFu) * ws.k_max + k];
            s0 = fma(x, (T)p.x, s0);
            s1 = fma(x, (T)p.y, s1);
        }
    } else {
        const double* r0 = ws.lt64 + (int64_t)(ws.k_max + 2 * k) * ws.G;
        const double* r1 = r0 + ws.G;
        for (int64_t pos = b; pos < e; ++pos) {
            const uint32_t en = ws.ent[pos];
            const T x = (T)(en >> 16);
            if (x == 0) continue;
            const int g = (int)(en & 0xFFFFu);
            s0 = fma(x, (T)r0[g], s0);
            s1 = fma(x, (T)r1[g], s1);
        }
    }
}

template <typename T>
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
    if (K <= 16) cluster_pass<T, 16>(ws, a, tab, i, valid, b, e, K, top);
    else if (K <= 32) cluster_pass<T, 32>(ws, a, tab, i, valid, b, e, K, top);
    else if (sizeof(T) == 4 && K <= 48) cluster_pass<T, 48>(ws, a, tab, i, valid, b, e, K, top);
    else cluster_pass<T, (sizeof(T) == 4 ? 64 : 32)>(ws, a, tab, i, valid, b, e, K, top);

    uint32_t flags = 0;
    if (valid && sizeof(T) == 4 && a.refine && K >= 2) {
        const float gap = (float)(top.v1 - top.v2);
        const float bnd = score_bound((float)top.a1, (float)top.p1, e - b) +
                          score_bound((float)top.a2, (float)top.p2, e - b);
        if (gap <= bnd || rel_margin((float)top.v1, (float)top.v2) < a.refine_tol) flags |= kRefineCluster;
    }

    // sub-cluster of the chosen cluster (eq. 8), always in FP64: two
    // products per entry, so its decision never needs re-scoring
    const int k = top.k1;
    const bool reset = valid ? ws.reset[k] != 0 : true;
    double s0, s1;
    sub_pass<double>(ws, reinterpret_cast<double*>(tab), b, e, K, k, valid && !reset, s0, s1);
    if (!valid) return;

    const int32_t c_old = a.c_old[i];
    const int s_old = a.cs_old[i] & 1;
    int sub;
    if (reset) {
        const Words w = philox(ws.seed, (uint32_t)i, 0u, a.step, kResub, 0u);
        sub = (int)(w.w[0] >> 31);
        if (a.dbg && K + 2 <= a.dbg_stride) {
            a.dbg[i * a.dbg_stride + K] = __builtin_nanf("");
            a.dbg[i * a.dbg_stride + K + 1] = __builtin_nanf("");
        }
    } else {
        const long long w0 = (long long)ws.nsub[2 * k] - ((c_old == k && s_old == 0) ? 1 : 0);
        const long long w1 = (long long)ws.nsub[2 * k + 1] - ((c_old == k && s_old == 1) ? 1 : 0);
        double lw0, lw1;
        if (w0 == 0 && w1 == 0) {
            lw0 = lw1 = 0.0;
        } else {
            lw0 = w0 > 0 ? log((double)w0) : -INFINITY;
            lw1 = w1 > 0 ? log((double)w1) : -INFINITY;
        }
        const Words w = philox(ws.seed, (uint32_t)i, 0u, a.step, kGumbelS, 0u);
        const double v0 = lw0 + s0 + gumbel_of<double>(w.w[0]);
        const double v1 = lw1 + s1 + gumbel_of<double>(w.w[1]);
        sub = v1 > v0 ? 1 : 0;
        if (a.dbg && K + 2 <= a.dbg_stride) {
            a.dbg[i * a.dbg_stride + K] = (float)s0;
            a.dbg[i * a.dbg_stride + K + 1] = (float)s1;
        }
    }
    a.c_new[i] = k;
    a.cs_new[i] = (uint8_t)sub;
    if (flags) {
        const int q = atomicAdd(&ws.st->n_refine, 1);
        if (q < ws.N) ws.refine[q] = (uint32_t)i | flags;
    }
}

void launch_assign_fp32(const Ws& ws, const AssignArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_assign_valu<float>, dim3((unsigned)((ws.N + kAssignThreads - 1) / kAssignThreads)),
                       dim3(kAssignThreads), 0, s, ws, a);
}

void launch_assign_fp64(const Ws& ws, const AssignArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_assign_valu<double>, dim3((unsigned)((ws.N + kAssignThreads - 1) / kAssignThreads)),
                       dim3(kAssignThreads), 0, s, ws, a);
}

// ---------------------------------------------------------------------------
// FP64 re-score of queued decisions: the cluster choice over all K (when
// flagged) and then the sub-cluster choice in the chosen cluster, with FP64
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
            double best = -INFINITY;
            int bk = 0;
            Words w{};
            for (int kk = 0; kk < K; ++kk) {
                if ((kk & 3) == 0) w = philox(ws.seed, (uint32_t)i, (uint32_t)(kk >> 2), a.step, kGumbelC, 0u);
                const double v = ws.logpi[kk] + row_dot64(ws, b, e, ws.lt64 + (int64_t)kk * ws.G) +
                                 gumbel_of<double>(w.w[kk & 3]);
                if (v > best) { best = v; bk = kk; }
            }
            k = bk;
        }
        int sub;
        if (ws.reset[k]) {
            const Words w = philox(ws.seed, (uint32_t)i, 0u, a.step, kResub, 0u);
            sub = (int)(w.w[0] >> 31);
        } else {
            const int32_t c_old = a.c_old[i];
            const int s_old = a.cs_old[i] & 1;
            const long long w0 = (long long)ws.nsub[2 * k] - ((c_old == k && s_old == 0) ? 1 : 0);
            const long long w1 = (long long)ws.nsub[2 * k + 1] - ((c_old == k && s_old == 1) ? 1 : 0);
            double lw0, lw1;
            if (w0 == 0 && w1 == 0) {
                lw0 = lw1 = 0.0;
            } else {
                lw0 = w0 > 0 ? log((double)w0) : -INFINITY;
                lw1 = w1 > 0 ? log((double)w1) : -INFINITY;
            }
            const double* r0 = ws.lt64 + (int64_t)(ws.k_max + 2 * k) * ws.G;
            const Words w = philox(ws.seed, (uint32_t)i, 0u, a.step, kGumbelS, 0u);
            const double v0 = lw0 + row_dot64(ws, b, e, r0) + gumbel_of<double>(w.w[0]);
            const double v1 = lw1 + row_dot64(ws, b, e, r0 + ws.G) + gumbel_of<double>(w.w[1]);
            sub = v1 > v0 ? 1 : 0;
        }
        a.c_new[i] = k;
        a.cs_new[i] = (uint8_t)sub;
        atomicAdd(&ws.st->counters[kCntRefined], 1ull);
    }
}

void launch_refine(const Ws& ws, const AssignArgs& a, hipStream_t s)
{
    int64_t blocks = (ws.N + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_refine, dim3((unsigned)blocks), dim3(256), 0, s, ws, a);
}

}  // namespace dpmm
