// substats.hip -- the sub-cluster draw (Section 2.3, eq. 8) fused with the
// integer sufficient statistics (step a4).
//
// After the cluster draw, the cells are counting-sorted by their new cluster
// (`perm`, offsets `grp_off`).  A workgroup takes ws.sub_cells consecutive
// sorted cells, i.e. one run (or a few) of a single cluster k.  For each run
// it stages delta_u = log thetabar_{k,1,u} - log thetabar_{k,0,u} (FP64) in
// LDS: the draw compares the two sub-cluster scores, and their difference is
// sum_u x_i^u delta_u, one product per entry.  Each wavefront takes 64 sorted
// cells at a time: one lane per cell first forms the cell's Philox words and
// FP32 Gumbel noise difference, then 8 lanes per cell, eight cells at a time,
// read the rows with 16-byte loads (ten per lane in flight: eight rows of up to
// 320 entries per round trip; the row reads bound the kernel, so the more rows
// in flight the better), form the FP64 difference (fixed-order reduction over
// the 8 lanes), draw cbar_i by Gumbel-max with weights
// nbar_{k,r} less the cell's own old membership, and add the row's counts to
// the LDS histogram of (k, cbar_i).  The two scores themselves are formed only
// for the debug dump.  The histograms are flushed with one 64-bit atomic per
// non-zero gene.  The matrix is read once for both jobs.
//
// When the next split/merge call is a random split (chain B, Section 2.4; its
// pass is a function of the seed and the step alone), the same pass also
// draws every cell's fair coin for it and builds the statistics of the coin
// halves of each cluster in a second pair of histograms, so that the random
// split needs no pass over the matrix of its own.
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

constexpr int kSubThreads = 256;
constexpr int kSubCellsMin = 256;       // sorted cells per workgroup, at least
constexpr int kSubStageGenes = 4096;     // delta staged in LDS up to this G
constexpr int kSubHistGenes = 8192;      // LDS histograms up to this G
constexpr int kSubLanes = 8;             // lanes per cell: eight cells of a wavefront read their rows together
constexpr int kStageBatch = 8;           // genes per thread whose delta loads are in flight together
constexpr int kSubLoads = 10;            // 16-byte loads per lane in flight: the first 320 entries of a row

// sum over the kSubLanes lanes of a cell, in a fixed order
__device__ inline double group_sum(double v)
{
    for (int o = kSubLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kSubLanes);
    return v;
}

// STAGE: delta in LDS; LHIST: histograms in LDS; DUMP: also form the two
// scores for the debug dump; SPLITQ: keep log p(cbar_i) for the split
// proposal term.  The flags are template arguments so that the loop over a
// row's entries is straight-line code.
template <bool STAGE, bool LHIST, bool DUMP, bool SPLITQ>
__global__ void __launch_bounds__(kSubThreads) __attribute__((amdgpu_waves_per_eu(3))) k_sub_stats(Ws ws, SubArgs a)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const int G = ws.G;
    constexpr bool stage = STAGE, lhist = LHIST, dump = DUMP;
    double* dl = reinterpret_cast<double*>(lds);                        // [G] delta if staged
    uint32_t* hist = reinterpret_cast<uint32_t*>(lds + (stage ? 8 * (size_t)G : 0));    // [2][G], then a spare slot per lane
    __shared__ uint32_t ncnt[2], ncnt2[2];
    const bool rs = a.rsplit != 0;
    uint32_t* hist2 = hist + 2 * G + 64;                                 // [2][G] coin halves, then a spare slot per lane
    if (blockIdx.x == 0 && threadIdx.x == 0) ws.st->rs_live = rs ? 1 : 0;
    const int K = ws.st->K;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t p0 = (int64_t)blockIdx.x * ws.sub_cells;
    const int64_t p1 = min(ws.N, p0 + ws.sub_cells);
    if (p0 >= p1) return;
    // first cluster whose run reaches p0
    int k = 0;
    {
        int lo = 0, hi = K;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (ws.grp_off[mid] <= p0) lo = mid;
            else hi = mid;
        }
        k = lo;
    }
    for (; k < K && ws.grp_off[k] < p1; ++k) {
        const int64_t r0 = max(p0, (int64_t)ws.grp_off[k]);
        const int64_t r1 = min(p1, (int64_t)ws.grp_off[k + 1]);
        if (r0 >= r1) continue;
        const bool reset = ws.reset[k] != 0;
        const double* g0 = ws.lt64 + (int64_t)(ws.k_max + 2 * k) * G;
        const double* g1 = g0 + G;
        __syncthreads();
        if (stage && !reset) {
            // kStageBatch genes per thread at a time, their loads issued together
            for (int u0 = threadIdx.x; u0 < G; u0 += kSubThreads * kStageBatch) {
                double h1[kStageBatch], h0[kStageBatch];
#pragma unroll
                for (int j = 0; j < kStageBatch; ++j) {
                    const int u = u0 + j * kSubThreads;
                    h1[j] = u < G ? g1[u] : 0.0;
                    h0[j] = u < G ? g0[u] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < kStageBatch; ++j) {
                    const int u = u0 + j * kSubThreads;
                    if (u < G) dl[u] = h1[j] - h0[j];
                }
            }
        }
        if (lhist)
            for (int u = threadIdx.x; u < 2 * G; u += kSubThreads) hist[u] = 0;
        if (lhist && rs)
            for (int u = threadIdx.x; u < 2 * G; u += kSubThreads) hist2[u] = 0;
        if (threadIdx.x < 2) ncnt[threadIdx.x] = ncnt2[threadIdx.x] = 0;
        __syncthreads();
        // log of the eq. 8 weights: nbar_{k,r}, less one when the cell was in (k, r)
        const SubWeights sw = sub_weights(ws.nsub_prev, k);
        // Each wavefront takes 64 sorted cells at a time.  First one lane per
        // cell forms what depends on the cell alone (its row descriptor, which
        // also carries its old membership, so that one load serves; the
        // Philox words and the FP32 noise difference);
        // then kSubLanes lanes per cell, 64 / kSubLanes cells at a time, read
        // the rows, and the per-cell values come by lane shuffles.
        const int grp = lane / kSubLanes;
        const int lg = lane % kSubLanes;
        for (int64_t base = r0 + 64 * wave; base < r1; base += 64 * (kSubThreads / 64)) {
            const int ncell = (int)min((int64_t)64, r1 - base);
            uint4 dsc = make_uint4(0, 0, 0, 0);
            float nd = 0.0f;      // FP32 Gumbel noise of sub-cluster 1 less that of 0
            int code = 0;         // reset: the fair draw; else 1 + old sub-label if the cell was in k, 0 if not
            int coin = 0;         // the cell's coin of the coming random split
            if (lane < ncell) {
                dsc = ws.srow[base + lane];
                const uint32_t i = dsc.x;
                if (rs) {
                    coin = (int)(philox(ws.seed, i, 0u, a.rs_step, kRSplit, 0u).w[0] >> 31);
                    ws.rbits[i] = (uint8_t)coin;
                }
                if (reset) {
                    code = (int)(philox(ws.seed, i, 0u, a.step, kResub, 0u).w[0] >> 31);
                } else {
                    nd = sub_noise(ws.seed, i, a.step, kGumbelS);
                    code = (int)(dsc.w >> kSrowOldShift);      // written by the sort
                }
            }
            for (int c0 = 0; c0 < ncell; c0 += 64 / kSubLanes) {
                const int src = c0 + grp;
                const bool live = src < ncell;
                const int64_t i = (int64_t)(uint32_t)__shfl((int)dsc.x, src);
                const int64_t b = (int64_t)(((uint64_t)(uint32_t)__shfl((int)dsc.z, src) << 32) |
                                            (uint32_t)__shfl((int)dsc.y, src));
                const uint32_t len = (uint32_t)__shfl((int)dsc.w, src) & kSrowLenMask;
                const int64_t e = live ? b + len : b;
                const float ndc = __shfl(nd, src);
                const int cc = __shfl(code, src);
                const int rc = __shfl(coin, src);
                int sub;
                double df = 0.0, s0 = 0.0, s1 = 0.0;
                double dd = 0.0;        // score of sub-cluster 1 less that of 0 (with the weights)
                // the first 4 kSubLanes kSubLoads (320) entries of the row
                // (nearly every row), all loads in flight together
                uint4 v[kSubLoads];
#pragma unroll
                for (int r = 0; r < kSubLoads; ++r) {
                    const int64_t q = b + 4 * lg + 4 * kSubLanes * r;
                    v[r] = q < e ? *reinterpret_cast<const uint4*>(ws.ent + q) : make_uint4(kPadEntry, kPadEntry, kPadEntry, kPadEntry);
                }
                auto dot = [&](const uint4& u) {
                    const uint32_t en[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint32_t x = en[j] >> 16;
                        if (!x) continue;
                        const int g = (int)(en[j] & 0xFFFFu);
                        df = fma((double)x, stage ? dl[g] : g1[g] - g0[g], df);
                        if (dump) {
                            s0 = fma((double)x, g0[g], s0);
                            s1 = fma((double)x, g1[g], s1);
                        }
                    }
                };
                if (reset) {
                    sub = cc;
                } else {
#pragma unroll
                    for (int r = 0; r < kSubLoads; ++r) dot(v[r]);
                    for (int64_t q = b + 4 * lg + 4 * kSubLanes * kSubLoads; q < e; q += 4 * kSubLanes) dot(*reinterpret_cast<const uint4*>(ws.ent + q));
                    df = group_sum(df);
                    if (dump) {
                        s0 = group_sum(s0);
                        s1 = group_sum(s1);
                    }
                    sub = sub_draw(ws.seed, (uint32_t)i, a.step, kGumbelS, sw, cc, ndc, df, &dd);
                }
                // statistics of (k, sub), from the registers where the row already is
                unsigned long long* grow = ws.ssub + (int64_t)(2 * k + sub) * G;
                auto add = [&](const uint4& u) {
                    const uint32_t en[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint32_t x = en[j] >> 16;
                        const uint32_t g = en[j] & 0xFFFFu;
                        if constexpr (LHIST) {
                            // a pad entry adds 0 to the lane's spare slot
                            atomicAdd(&hist[x ? sub * G + g : 2 * G + lane], x);
                            if (rs) atomicAdd(&hist2[x ? rc * G + g : 2 * G + lane], x);
                        } else {
                            if (!x) continue;
                            atomicAdd(&grow[g], (unsigned long long)x);
                            if (rs) atomicAdd(&ws.rssub[(int64_t)(2 * k + rc) * G + g], (unsigned long long)x);
                        }
                    }
                };
#pragma unroll
                for (int r = 0; r < kSubLoads; ++r) add(v[r]);
                for (int64_t q = b + 4 * lg + 4 * kSubLanes * kSubLoads; q < e; q += 4 * kSubLanes) add(*reinterpret_cast<const uint4*>(ws.ent + q));
                if (lg == 0 && live) {
                    atomicAdd(&ncnt[sub], 1u);
                    if (rs) atomicAdd(&ncnt2[rc], 1u);
                    a.cs_new[i] = (uint8_t)sub;
                    if constexpr (SPLITQ) {
                        // log p(cbar_i) of eq. 8 for the split proposal term: a
                        // two-way softmax of the scores, whose difference is dd
                        ws.subdd[i] = reset ? __builtin_nan("") : dd;
                    }
                    if (a.dbg && K + 2 <= a.dbg_stride) {
                        put_dbg(a.dbg, a.dbg64, i * a.dbg_stride + K, reset ? __builtin_nan("") : s0);
                        put_dbg(a.dbg, a.dbg64, i * a.dbg_stride + K + 1, reset ? __builtin_nan("") : s1);
                    }
                }
            }
        }
        __syncthreads();
        if (lhist) {
            unsigned long long* row = ws.ssub + (int64_t)(2 * k) * G;
            for (int u = threadIdx.x; u < 2 * G; u += kSubThreads) {
                const uint32_t v = hist[u];
                if (v) atomicAdd(&row[u], (unsigned long long)v);
            }
        }
        if (lhist && rs) {
            unsigned long long* row = ws.rssub + (int64_t)(2 * k) * G;
            for (int u = threadIdx.x; u < 2 * G; u += kSubThreads) {
                const uint32_t v = hist2[u];
                if (v) atomicAdd(&row[u], (unsigned long long)v);
            }
        }
        if (threadIdx.x < 2 && ncnt[threadIdx.x])
            atomicAdd(&ws.nsub[2 * k + threadIdx.x], (unsigned long long)ncnt[threadIdx.x]);
        if (rs && threadIdx.x < 2 && ncnt2[threadIdx.x])
            atomicAdd(&ws.rnsub[2 * k + threadIdx.x], (unsigned long long)ncnt2[threadIdx.x]);
    }
}

static size_t sub_stats_lds(int G, bool rs)
{
    size_t lds = 0;
    if (G <= kSubStageGenes) lds += 8 * (size_t)G;
    if (G <= kSubHistGenes) lds += (rs ? 2 : 1) * (8 * (size_t)G + 4 * 64);   // + a spare slot per lane
    return lds;
}

using SubKernel = void (*)(Ws, SubArgs);

template <bool SPLITQ>
static SubKernel sub_stats_variant(int G, bool dump)
{
    if (G <= kSubStageGenes)
        return dump ? k_sub_stats<true, true, true, SPLITQ> : k_sub_stats<true, true, false, SPLITQ>;
    if (G <= kSubHistGenes)
        return dump ? k_sub_stats<false, true, true, SPLITQ> : k_sub_stats<false, true, false, SPLITQ>;
    return dump ? k_sub_stats<false, false, true, SPLITQ> : k_sub_stats<false, false, false, SPLITQ>;
}

static SubKernel sub_stats_kernel(int G, bool dump, bool split_q)
{
    return split_q ? sub_stats_variant<true>(G, dump) : sub_stats_variant<false>(G, dump);
}

// Sorted cells per workgroup: the grid fills the device's resident workgroup
// slots once (a second, partial round would leave most of the device idle).
hipError_t sub_stats_cells(int64_t N, int G, int32_t* cells)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipSuccess;
    // allow every variant the LDS of the pass with the coin halves
    for (int v = 0; v < 4 && e == hipSuccess; ++v)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(sub_stats_kernel(G, v & 1, v >> 1)),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sub_stats_lds(G, true));
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(sub_stats_kernel(G, false, false)),
                                                         kSubThreads, sub_stats_lds(G, false));
    if (e != hipSuccess) return e;
    const int64_t slots = (int64_t)(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
    int64_t c = (N + slots - 1) / slots;
    c = (c + 63) / 64 * 64;
    *cells = (int32_t)(c < kSubCellsMin ? kSubCellsMin : c);
    return hipSuccess;
}

void launch_sub_stats(const Ws& ws, const SubArgs& a, hipStream_t s)
{
    // the counts (and, with rsplit, the coin halves') were cleared by the
    // redraw of the same sweep (k_redraw_norm)
    launch_sort(ws, a.c_new, a.cs_old, 1, s, true, a.c_old);
    hipLaunchKernelGGL(sub_stats_kernel(ws.G, a.dbg != nullptr, ws.subdd != nullptr), dim3((unsigned)((ws.N + ws.sub_cells - 1) / ws.sub_cells)), dim3(kSubThreads),
                       sub_stats_lds(ws.G, a.rsplit != 0), s, ws, a);
}

}  // namespace dpmm
