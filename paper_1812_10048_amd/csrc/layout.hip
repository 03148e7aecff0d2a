// layout.hip -- the cluster-sorted copy of the count matrix read by the
// matrix-core kernel (split-BF16), rebuilt from the labels when the partition
// has changed.
//
// The profiles theta_k of droplet data put most of a cluster's counts on a few
// hundred genes, and which genes those are differs from cluster to cluster.
// So the copy is built per cluster: the cells of cluster L (labels at build
// time) are taken in blocks of kBlkCells (a cluster's last block is padded
// with empty slots), and the genes are renumbered for L by decreasing count
// s_{L,u} (the cluster's sufficient statistics).  In that order a block's
// counts crowd into the first few chunks of kBlkGenes genes.  The first D_b
// chunks of block b are stored dense, one byte per (cell, gene), in the order
// of the matrix-core fragments; every other entry (a gene past those chunks,
// or a count above 255) is a tail entry of its cell, (gene | count << 16).
// D_b (at most kLayDmax) minimises the block's cost, 16 KiB per dense chunk
// against kTailCost per tail entry.  A count above 255 on one of the first
// kPlaneGenes places (the cluster's top genes, where such counts crowd) is
// split when D_b >= 1: its low byte goes to chunk 0, its high byte to a high
// plane (one more chunk slot after the D_b, of which it fills the first half:
// the A fragments of one k-step, 8 bytes per lane; scored with weight 256),
// and 256 x the high byte stays in the cell's tail, last, for the sub-cluster
// pass and the statistics (lay_hcnt of them per slot; lay_bh[b] = 1 when the
// block has the plane).
//
// The copy only decides how each cell's log-likelihoods are summed; any cell
// in any block is scored exactly the same way, so the copy may lag behind the
// labels.  It is rebuilt at init and at dpmm_set_state, and by the sweeps when
// the partition has changed structurally (a cluster appeared, disappeared or
// was renumbered); the build kernels then run gated on a device flag.
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

constexpr int kLayThreads = kBlkCells;        // one thread per block slot
constexpr int kRankThreads = 1024;
constexpr int kRankMaxGenes = 8192;           // genes renumbered per cluster up to this G

__device__ inline bool lay_gate(const Ws& ws, int gated) { return !gated || ws.st->lay_go; }

// Decide whether the copy is stale: the partition changed structurally since
// it was built (K differs, or labels were renumbered).
__global__ void k_lay_decide(Ws ws, int force)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    DevState* st = ws.st;
    st->lay_go = (force || st->K != st->lay_K || st->relabels != st->lay_relabels) ? 1 : 0;
}

// One thread: the blocks of each cluster (from the sort's group offsets), the
// block -> (cluster, first sorted cell, cells) map, and the number of blocks.
__global__ void k_lay_plan(Ws ws, int gated)
{
    if (threadIdx.x != 0 || blockIdx.x != 0 || !lay_gate(ws, gated)) return;
    const int K = ws.st->K;
    int b = 0, x = 0;
    for (int k = 0; k < K; ++k) {
        const int beg = ws.grp_off[k], end = ws.grp_off[k + 1];
        ws.lay_bbeg[k] = b;
        ws.lay_sbeg[k] = x;
        const int b_first = b;
        for (int p = beg; p < end && b < ws.nblk_cap; p += kBlkCells, ++b) {
            ws.lay_kc[b] = k;
            ws.lay_pbeg[b] = p;
            ws.lay_pcnt[b] = min(kBlkCells, end - p);
        }
        x += (b - b_first + kSpanBlocks - 1) / kSpanBlocks;
    }
    ws.lay_bbeg[K] = b;
    ws.lay_sbeg[K] = x;
    ws.st->lay_nblk = b;
    ws.st->lay_K = K;
    ws.st->lay_relabels = ws.st->relabels;
}

// One workgroup per cluster: the genes in decreasing order of the cluster's
// count s_{k,0,u} + s_{k,1,u}, ties by gene (a bitonic sort of 64-bit keys in
// LDS).  rank[k][u] is gene u's place, gene[k][j] the gene at place j (first
// kLayDmax chunks).  Past kRankMaxGenes genes the order is the identity.
__global__ void __launch_bounds__(kRankThreads) k_lay_ranks(Ws ws, int gated)
{
    extern __shared__ unsigned long long keys[];
    if (!lay_gate(ws, gated)) return;
    const int K = ws.st->K;
    const int k = blockIdx.x;
    if (k >= K) return;
    const int G = ws.G;
    uint16_t* rank = ws.lay_rank + (int64_t)k * G;
    uint16_t* gene = ws.lay_gene + (int64_t)k * kLayDmax * kBlkGenes;
    if (G > kRankMaxGenes) {
        for (int u = threadIdx.x; u < G; u += kRankThreads) rank[u] = (uint16_t)u;
        for (int j = threadIdx.x; j < kLayDmax * kBlkGenes; j += kRankThreads) gene[j] = (uint16_t)(j < G ? j : 0);
        return;
    }
    int n = 1;
    while (n < G) n <<= 1;
    const unsigned long long* s0 = ws.ssub + (int64_t)(2 * k) * G;
    const unsigned long long* s1 = s0 + G;
    constexpr unsigned long long kMaxCount = (1ull << 47) - 1ull;
    for (int u = threadIdx.x; u < n; u += kRankThreads) {
        unsigned long long v = 0;
        if (u < G) {
            const unsigned long long c = s0[u] + s1[u];
            // larger count first, then smaller gene: descending key order
            v = ((c < kMaxCount ? c : kMaxCount) << 16) | (unsigned long long)(0xFFFFu - (unsigned)u);
            v += 1ull << 63;      // genes sort above the padding keys (0)
        }
        keys[u] = v;
    }
    __syncthreads();
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < n; i += kRankThreads) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;     // descending runs first
                    const unsigned long long a = keys[i], b = keys[j];
                    if (desc ? a < b : a > b) {
                        keys[i] = b;
                        keys[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int j = threadIdx.x; j < G; j += kRankThreads) {
        const int u = (int)(0xFFFFu - (unsigned)(keys[j] & 0xFFFFull));
        rank[u] = (uint16_t)j;
        if (j < kLayDmax * kBlkGenes) gene[j] = (uint16_t)u;
    }
    for (int j = G + threadIdx.x; j < kLayDmax * kBlkGenes; j += kRankThreads) gene[j] = 0;
}

// One workgroup per block: the cell of each slot, its number of entries, the
// block's dense chunk count D_b and each slot's number of tail entries (into
// the arrays that the scans turn into offsets).
__global__ void __launch_bounds__(kLayThreads) k_lay_count(Ws ws, int gated)
{
    __shared__ uint32_t hist[kLayDmax];
    __shared__ uint32_t s_D;
    if (!lay_gate(ws, gated)) return;
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t slot = (int64_t)b * kBlkCells + t;
    if (b >= ws.st->lay_nblk) {
        if (t == 0) {
            ws.lay_doff[b] = 0;
            ws.lay_bh[b] = 0;
        }
        ws.lay_toff[slot] = 0;
        ws.lay_cell[slot] = -1;
        ws.lay_nnz[slot] = 0;
        ws.lay_hcnt[slot] = 0;
        return;
    }
    if (t < kLayDmax) hist[t] = 0;
    __syncthreads();
    const int kc = ws.lay_kc[b];
    const int cell = t < ws.lay_pcnt[b] ? ws.perm[ws.lay_pbeg[b] + t] : -1;
    const uint16_t* rank = ws.lay_rank + (int64_t)kc * ws.G;
    const int64_t rb = cell >= 0 ? ws.roff[cell] : 0, re = cell >= 0 ? ws.roff[cell + 1] : 0;
    // pass 1: the block's entries per chunk of the cluster's gene order
    // (rows are padded to 16 bytes, so they are read four entries at a time)
    uint32_t nnz = 0;
    for (int64_t p = rb; p < re; p += 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(ws.ent + p);
        const uint32_t en[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t x = en[q] >> 16;
            const uint32_t g = en[q] & 0xFFFFu;
            if (!x || g >= (uint32_t)ws.G) continue;
            ++nnz;
            const uint32_t ch = rank[g] / kBlkGenes;
            if (x < 256u && ch < (uint32_t)kLayDmax) atomicAdd(&hist[ch], 1u);
        }
    }
    __syncthreads();
    if (t == 0) {
        // cost of D dense chunks: 16 KiB each, plus kTailCost per entry not
        // in them
        long long best = 0, cost = 0;
        uint32_t D = 0;
        for (int d = 1; d <= kLayDmax; ++d) {
            cost += (long long)kBlkCells * kBlkGenes - kTailCost * (long long)hist[d - 1];
            if (cost < best) {
                best = cost;
                D = (uint32_t)d;
            }
        }
        s_D = D;
    }
    __syncthreads();
    // pass 2: the slot's entries that stay out of the dense chunks, and its
    // counts above 255 on chunk 0's first kPlaneGenes places (split by the high
    // plane)
    const uint32_t lim = s_D * kBlkGenes;
    uint32_t dense = 0, big = 0;
    for (int64_t p = rb; p < re; p += 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(ws.ent + p);
        const uint32_t en[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t x = en[q] >> 16;
            const uint32_t g = en[q] & 0xFFFFu;
            if (!x || g >= (uint32_t)ws.G) continue;
            const uint32_t rk = rank[g];
            if (x < 256u && rk < lim) ++dense;
            else if (x >= 256u && rk < (uint32_t)kPlaneGenes && lim > 0) ++big;
        }
    }
    // the plane when any slot of the block has such a count
    const int H = __syncthreads_or(big > 0);
    if (t == 0) {
        ws.lay_doff[b] = s_D + (uint32_t)H;
        ws.lay_bh[b] = (uint8_t)H;
    }
    ws.lay_cell[slot] = cell;
    // (a split count is two products, of its low and its high byte)
    ws.lay_nnz[slot] = (uint16_t)min(nnz + big, 65535u);
    ws.lay_hcnt[slot] = (uint8_t)big;              // at most kPlaneGenes
    ws.lay_toff[slot] = (int64_t)(nnz - dense);
}

// Byte of (slot, place jj in chunk j) in the block's dense chunks: fragment
// order of v_mfma_f32_16x16x32_bf16's A operand, 16 bytes per lane holding
// the two k-steps of its row, lanes of a row tile contiguous.
__device__ inline uint32_t dense_byte(int slot, int j, int jj)
{
    const int w = slot >> 6, m = (slot >> 4) & 3, r = slot & 15;
    const int s = (jj >> 5) & 1, q = (jj >> 3) & 3, e = jj & 7;
    const int lane = 16 * q + r;
    return (uint32_t)j * kDenseChunkBytes + (uint32_t)(((w * 4 + m) * 64 + lane) * 16 + s * 8 + e);
}

// Byte of (slot, place jj < kPlaneGenes) in the high plane at chunk slot j:
// the same fragment order for the one k-step, 8 bytes per lane.
__device__ inline uint32_t plane_byte(int slot, int j, int jj)
{
    const int rt = slot >> 4, r = slot & 15;
    const int q = (jj >> 3) & 3, e = jj & 7;
    return (uint32_t)j * kDenseChunkBytes + (uint32_t)((rt * 64 + 16 * q + r) * 8 + e);
}

// One workgroup per block: the dense chunks assembled in LDS and written out
// with 16-byte stores; the tail entries of each slot in row order.
__global__ void __launch_bounds__(kLayThreads) k_lay_fill(Ws ws, int gated)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t tile[];     // [kLayDmax + 1][16 KiB]
    if (!lay_gate(ws, gated)) return;
    const int b = blockIdx.x;
    if (b >= ws.st->lay_nblk) return;
    const int t = threadIdx.x;
    const int H = ws.lay_bh[b];
    const int DT = (int)(ws.lay_doff[b + 1] - ws.lay_doff[b]);     // dense chunks and the plane
    const int D = DT - H;
    uint4* t4 = reinterpret_cast<uint4*>(tile);
    for (int q = t; q < DT * kDenseChunkBytes / 16; q += kLayThreads) t4[q] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    const int64_t slot = (int64_t)b * kBlkCells + t;
    const int cell = ws.lay_cell[slot];
    const int kc = ws.lay_kc[b];
    const uint16_t* rank = ws.lay_rank + (int64_t)kc * ws.G;
    if (cell >= 0) {
        // the tail entries in row order, then the high bytes' (256 x hi) last
        int64_t w = ws.lay_toff[slot];
        int64_t wh = ws.lay_toff[slot + 1] - ws.lay_hcnt[slot];
        const uint32_t lim = (uint32_t)D * kBlkGenes;
        for (int64_t p = ws.roff[cell]; p < ws.roff[cell + 1]; p += 4) {
            const uint4 v = *reinterpret_cast<const uint4*>(ws.ent + p);
            const uint32_t ent4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t en = ent4[q];
                const uint32_t x = en >> 16;
                const uint32_t g = en & 0xFFFFu;
                if (!x || g >= (uint32_t)ws.G) continue;
                const uint32_t rk = rank[g];
                if (x < 256u && rk < lim) {
                    tile[dense_byte(t, rk / kBlkGenes, rk % kBlkGenes)] = (uint8_t)x;
                } else if (H && x >= 256u && rk < (uint32_t)kPlaneGenes) {
                    tile[dense_byte(t, 0, rk)] = (uint8_t)(x & 0xFFu);
                    tile[plane_byte(t, D, rk)] = (uint8_t)(x >> 8);
                    ws.lay_tail[wh++] = g | ((x & 0xFF00u) << 16);
                } else {
                    ws.lay_tail[w++] = en;
                }
            }
        }
    }
    __syncthreads();
    uint4* out = reinterpret_cast<uint4*>(ws.lay_dense + ws.lay_doff[b] * kDenseChunkBytes);
    for (int q = t; q < DT * kDenseChunkBytes / 16; q += kLayThreads) out[q] = t4[q];
}

hipError_t configure_layout()
{
    hipError_t e = hipFuncSetAttribute((const void*)k_lay_fill, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)((kLayDmax + 1) * kDenseChunkBytes));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_lay_ranks, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(unsigned long long) * kRankMaxGenes));
    return e;
}

// Rebuild the copy from the labels c.  force: unconditionally (init,
// dpmm_set_state); else only when k_lay_decide finds it stale, every kernel
// being gated on that decision.
void launch_relayout(const Ws& ws, const int32_t* c, int64_t* tile_sums, int force, hipStream_t s)
{
    const int gated = force ? 0 : 1;
    hipLaunchKernelGGL(k_lay_decide, dim3(1), dim3(64), 0, s, ws, force);
    launch_sort(ws, c, nullptr, 1, s, false, nullptr, gated ? &ws.st->lay_go : nullptr);
    hipLaunchKernelGGL(k_lay_plan, dim3(1), dim3(64), 0, s, ws, gated);
    int n = 1;
    while (n < ws.G) n <<= 1;
    const size_t rank_lds = ws.G > kRankMaxGenes ? 0 : sizeof(unsigned long long) * (size_t)n;
    hipLaunchKernelGGL(k_lay_ranks, dim3((unsigned)ws.k_max), dim3(kRankThreads), rank_lds, s, ws, gated);
    hipLaunchKernelGGL(k_lay_count, dim3((unsigned)ws.nblk_cap), dim3(kLayThreads), 0, s, ws, gated);
    launch_exclusive_scan(ws.lay_doff, ws.nblk_cap, tile_sums, s, gated ? &ws.st->lay_go : nullptr);
    launch_exclusive_scan(ws.lay_toff, (int64_t)ws.nblk_cap * kBlkCells, tile_sums, s,
                          gated ? &ws.st->lay_go : nullptr);
    hipLaunchKernelGGL(k_lay_fill, dim3((unsigned)ws.nblk_cap), dim3(kLayThreads), (kLayDmax + 1) * kDenseChunkBytes, s, ws,
                       gated);
}

// The sub-cluster score difference of layout cluster L in fixed point, for
// the integer matrix-core sums of the sub-cluster pass (laysub.hip):
// delta_p = log thetabar_{L,1,u} - log thetabar_{L,0,u} at place p (gene u of
// L's order), v_p = rint(delta_p 2^E) with E = 54 - e_max (|delta_p| <
// 2^e_max for all p < kLayDmax kBlkGenes, so |v_p| <= 2^54), written as seven
// base-256 digits in -128 .. 127: v_p = sum_k d_{p,k} 256^k.  lay_lim holds
// the digits as the A operand of v_mfma_i32_16x16x32_i8 (row k, k-group g,
// 8 consecutive places), lay_dS[L][D][k] the digit sums over the first D
// chunks and lay_dE[L] = E; lay_dfull[L] holds delta_u gene-major (for the
// tail entries) and lay_sw[L] the weights of the draw (sub_weights).  The
// digits also go to columns K .. K + kSubDigits - 1 of L's hi table in BF16
// (exact: integers of at most 8 bits; the lo table is 0 there), so that the
// matrix-core cluster draw forms the digit sums sum_p x_p d_{p,k} as extra
// score columns, exactly in FP32 (every partial sum is an integer below
// 512 x 255 x 128 < 2^24).  Block L of k_lay_btab (256 threads), for every L
// of the copy that is a live, non-reset cluster.
// BF16 bits of a small integer (|v| <= 128: exact)
__device__ inline uint16_t bf16_of_int(int v) { return (uint16_t)(__float_as_uint((float)v) >> 16); }

__device__ inline void lay_dtab(const Ws& ws, int L, int K, int KL)
{
    constexpr int R = kLayDmax * kBlkGenes;
    constexpr int kNoExp = -(1 << 30);         // no non-zero difference
    __shared__ int8_t dig[R][8];
    __shared__ int red[4];
    const int t = threadIdx.x;
    const int G = ws.G;
    const double* g0 = ws.lt64 + (int64_t)(ws.k_max + 2 * L) * G;
    const double* g1 = g0 + G;
    // L's gene order is loaded before the checks (L < k_max: in the table)
    int ug[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) ug[h] = ws.lay_gene[(int64_t)L * R + t + 256 * h];
    if (L >= KL || L >= K || ws.reset[L]) return;
    for (int u = t; u < G; u += 256) ws.lay_dfull[(int64_t)L * G + u] = g1[u] - g0[u];
    if (t == 0) {
        const SubWeights w = sub_weights(ws.nsub_prev, L);
        double* o = ws.lay_sw + 4 * (int64_t)L;
        o[0] = w.l0;
        o[1] = w.l0m;
        o[2] = w.l1;
        o[3] = w.l1m;
    }
    double d[2];
    int e = kNoExp;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int u = ug[h];
        d[h] = g1[u] - g0[u];
        if (d[h] != 0.0) {
            int ex;
            frexp(d[h], &ex);
            e = max(e, ex);
        }
    }
    for (int o = 32; o > 0; o >>= 1) e = max(e, __shfl_xor(e, o, 64));
    if ((t & 63) == 0) red[t >> 6] = e;
    __syncthreads();
    const int emax = max(max(red[0], red[1]), max(red[2], red[3]));
    const int E = emax == kNoExp ? 0 : 54 - emax;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        long long v = (long long)rint(ldexp(d[h], E));
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const int dk = (int)(int8_t)(uint8_t)(v & 0xFF);
            dig[t + 256 * h][k] = (int8_t)dk;
            v = (v - dk) >> 8;
        }
        dig[t + 256 * h][7] = 0;
    }
    __syncthreads();
    // the digit columns of L's hi / lo tables
    for (int q = t; q < kSubDigits * R; q += 256) {
        const int k = q / R, p = q - k * R;
        const int64_t at = ((int64_t)L * ws.lay_cols + K + k) * R + p;
        ws.lay_bhi[at] = bf16_of_int(dig[p][k]);
        ws.lay_blo[at] = 0;
    }
    // word (j, s, k, g): digit k of places 64 j + 32 s + 8 g .. + 7
    for (int w = t; w < kLayDmax * 2 * 8 * 4; w += 256) {
        const int g = w & 3, k = (w >> 2) & 7, s = (w >> 5) & 1, j = w >> 6;
        const int p0 = 64 * j + 32 * s + 8 * g;
        uint64_t word = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) word |= (uint64_t)(uint8_t)dig[p0 + b][k] << (8 * b);
        ws.lay_lim[(int64_t)L * (kLayDmax * 2 * 8 * 4) + w] = word;
    }
    // digit sums per chunk, then over the first D chunks
    __shared__ int csum[kLayDmax][8];
    if (t < kLayDmax * 8) {
        const int j = t >> 3, k = t & 7;
        int sum = 0;
        for (int p = 0; p < kBlkGenes; ++p) sum += dig[64 * j + p][k];
        csum[j][k] = sum;
    }
    __syncthreads();
    if (t < 8) {
        int acc = 0;
        int32_t* out = ws.lay_dS + (int64_t)L * (kLayDmax + 1) * 8;
        out[t] = 0;
        for (int j = 0; j < kLayDmax; ++j) {
            acc += csum[j][t];
            out[(j + 1) * 8 + t] = acc;
        }
        if (t == 0) ws.lay_dE[L] = E;
    }
}

// After every redraw: the hi/lo tables of log theta (split-BF16, cluster-major
// [k][Gpad]) with the genes in each layout cluster's order, for the first
// kLayDmax chunks: tab[L][col][j] = table[col][gene_L[j]], zero for the
// columns past K that the kernel's last column tile reads.  That kernel reads
// columns below K + kSubDigits rounded up to its column group (at most 64
// columns), so the columns from K + kSubDigits + 63 on are left as they are.
// The first k_max blocks write the fixed-point difference tables above
// instead.
__global__ void __launch_bounds__(256) k_lay_btab(Ws ws, int kd)
{
    const int K = ws.st->K;
    const int KL = ws.st->lay_K;
    const int R = kLayDmax * kBlkGenes;
    if ((int)blockIdx.x < kd) {
        // the first kd workgroups: clusters x, x + kd, ... (kd from a recent K)
        for (int L = blockIdx.x; L < KL && L < K; L += kd) {
            __syncthreads();               // (the LDS tables of the last cluster are read)
            lay_dtab(ws, L, K, KL);
        }
        return;
    }
    const int ncol = min(ws.lay_cols, K + kSubDigits + 63);
    const int64_t n = (int64_t)KL * ncol * R;
    const int64_t stride = (int64_t)(gridDim.x - kd) * blockDim.x;
    // (the digit columns of live, non-reset clusters are lay_dtab's)
    for (int64_t q = (int64_t)(blockIdx.x - kd) * blockDim.x + threadIdx.x; q < n; q += stride) {
        const int j = (int)(q % R);
        const int64_t lc = q / R;
        const int col = (int)(lc % ncol);
        const int L = (int)(lc / ncol);
        if (col >= K && col < K + kSubDigits && L < K && !ws.reset[L]) continue;
        uint16_t hi = 0, lo = 0;
        if (col < K) {
            const int64_t at = (int64_t)col * ws.Gpad + ws.lay_gene[(int64_t)L * R + j];
            hi = ws.lhi[at];
            lo = ws.llo[at];
        }
        const int64_t o = ((int64_t)L * ws.lay_cols + col) * R + j;
        ws.lay_bhi[o] = hi;
        ws.lay_blo[o] = lo;
    }
}

void launch_lay_btab(const Ws& ws, int k_guess, hipStream_t s)
{
    const int kd = k_guess > 0 && k_guess < ws.k_max ? k_guess : ws.k_max;
    const int64_t n = (int64_t)kd * (kd + kSubDigits + 63) * kLayDmax * kBlkGenes;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_lay_btab, dim3((unsigned)(blocks + kd)), dim3(256), 0, s, ws, kd);
}

}  // namespace dpmm
