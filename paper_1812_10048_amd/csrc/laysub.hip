// laysub.hip -- the sub-cluster draw (Section 2.3, eq. 8) and the integer
// sufficient statistics (step a4) of a split-BF16 sweep, over the
// cluster-sorted copy of the counts (layout.hip) instead of the packed matrix.
//
// A workgroup of 8 wavefronts takes one block of the copy, with layout
// cluster L; wavefront w owns the block's row tiles 2w and 2w + 1 (32 cells),
// whose dense bytes are stored as the A fragments of the matrix-core products
// (lane l: cell l % 16 of the tile, places 8 (l / 16) .. + 7 and
// 32 + 8 (l / 16) .. + 7 of each chunk of 64 places).  The block's cells whose
// new label is L (nearly all of them once the chain has settled) are drawn
// here; any other cell of the block goes to a queue that k_mov_span serves
// from the packed matrix, exactly as the packed-matrix pass would.  After the
// workgroup has staged what depends on L, each wavefront works on its own,
// with no further barrier until the block's histogram is written:
//   1. Each lane loads its fragments of both tiles, all chunks in flight at
//      once, keeps them in registers and forms the FP64 sums of x_u delta_u
//      over its 16 places per chunk, delta_u = log thetabar_{L,1,u} -
//      log thetabar_{L,0,u} staged in LDS in L's gene order; the four lanes
//      of a cell split its tail entries, and their sums are added in a fixed
//      pattern that gives all four the same value.
//   2. The draw itself (sub_draw, shared with the packed-matrix pass), taken
//      by the four lanes of a cell alike.
//   3. Statistics on the matrix cores, in 8-bit integers with 32-bit sums
//      (exact).  The fragments hold a cell's genes along k, the statistics
//      sum over cells: a product with a 0/1 selection matrix (one 1 per
//      column) turns the counts of 16 places of a tile into the layout where
//      each lane holds one place of four cells; packed as bytes, the counts of
//      the wavefront's 32 cells then multiply the 0/1 rows "cell of L in
//      sub-cluster 0", "... 1" (and "coin 0", "coin 1" of a random split
//      coming next) over those cells.  The signed operands take x - 128 and
//      the row's cell count times 128 is added back.  The sums go to a
//      per-block LDS histogram over (row, gene), together with the tail
//      entries (a count above 255 is a tail entry too, and those crowd on a
//      cluster's top genes).  Each block writes its whole histogram to
//      lay_part; k_mov_span adds them over spans of consecutive blocks of a
//      cluster and adds the span sums to the statistics: device-scope 64-bit
//      atomics from every cell (or every block) on a cluster's few hot
//      addresses would serialise.  (Past kLsHistWords histogram words, the
//      sums go to the statistics with atomics instead.)
#include "dpmm_common.hpp"
#include "kernels.hpp"
#include "laystats.hpp"

namespace dpmm {

constexpr int kLsThreads = 2 * kBlkCells;     // 8 wavefronts of 32 cells
constexpr int kMovGroups = kPlaces / 8;        // cells per workgroup pass of the queue (8 lanes each)
constexpr int kMovLanes = 8;
constexpr int kRedSpan = kSpanBlocks;

template <bool DUMP, bool SPLITQ>
__global__ void __launch_bounds__(kLsThreads) __attribute__((amdgpu_waves_per_eu(DUMP ? 2 : 8)))
k_lay_sub(Ws ws, SubArgs a)
{
    __shared__ double dl[DUMP ? kPlaces : 1];              // delta in L's gene order (dump)
    __shared__ uint64_t s_lim[DUMP ? 1 : kPlaces];         // its fixed-point digits (lay_lim of L)
    __shared__ double tl0[DUMP ? kPlaces : 1], tl1[DUMP ? kPlaces : 1];   // the two rows themselves (dump)
    __shared__ uint32_t phist[kPartRows][kPlaces];         // count sums per (row, place of L)
    __shared__ uint32_t ncnt[2], ncnt2[2];

    const bool rs = a.rsplit != 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) ws.st->rs_live = rs ? 1 : 0;
    const int b = blockIdx.x;
    if (b >= ws.st->lay_nblk) return;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int r = lane & 15;                   // the lane's row of its two tiles
    const int g = lane >> 4;                   // and its k-group
    const int L = ws.lay_kc[b];
    const int K = ws.st->K;
    const int G = ws.G;
    const int64_t d0 = ws.lay_doff[b];
    // (the high plane after the D dense chunks is for the cluster scores; the
    // high parts of those counts are in the tail entries here)
    const int D = (int)(ws.lay_doff[b + 1] - d0) - ws.lay_bh[b];
    const bool reset = L < K ? ws.reset[L] != 0 : true;
    const double* g0 = ws.lt64 + (int64_t)(ws.k_max + 2 * (L < K ? L : 0)) * G;
    const double* g1 = g0 + G;

    // the lane's fragments of row tiles 2w, 2w + 1: + j chunk + m 1 KiB
    const uint8_t* dense = ws.lay_dense + d0 * kDenseChunkBytes;   // uniform base
    const uint32_t doff = (uint32_t)((wave * 2) * 64 + lane) * 16;
    // chunk 0 in flight while the block stages (a block has at least one chunk
    // or none of its cells has a dense byte; chunk 0 of an empty block is never read)
    uint4 f0 = make_uint4(0, 0, 0, 0), f1 = f0;
    if (D > 0) {
        f0 = frag(dense, doff, 0, 0);
        f1 = frag(dense, doff, 0, 1);
    }
    // the lane's cells, their tail ranges and old labels, and (before the
    // barrier, so that the chain of loads overlaps the staging) the lane's
    // first tail entry of each with its difference
    int cell[2], ocode[2];
    bool stay[2];
    int64_t tb[2], te[2];
    uint32_t en0[2];
    int rk0[2];
    double dt0[2];
    const double* dfull = ws.lay_dfull + (int64_t)(L < K ? L : 0) * G;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int64_t slot = (int64_t)b * kBlkCells + 32 * wave + 16 * m + r;
        cell[m] = ws.lay_cell[slot];
        tb[m] = ws.lay_toff[slot];
        te[m] = ws.lay_toff[slot + 1];
        // (the loads below depend only on the slot, not on whether the cell
        // stays, so that they are in flight together)
        const int ci = cell[m] >= 0 ? cell[m] : 0;
        const int cn = a.c_new[ci], co = a.c_old[ci], so = a.cs_old[ci];
        const uint32_t en = cell[m] >= 0 && L < K && tb[m] + g < te[m] ? ws.lay_tail[tb[m] + g] : 0u;
        stay[m] = cell[m] >= 0 && L < K && cn == L;
        ocode[m] = stay[m] && co == L ? 1 + (so & 1) : 0;
        en0[m] = stay[m] ? en : 0u;                      // (an entry's count is >= 1)
        dt0[m] = !DUMP && !reset && en ? dfull[en & 0xFFFFu] : 0.0;
        rk0[m] = en ? ws.lay_rank[(int64_t)L * G + (en & 0xFFFFu)] : 0;
        if (g == 0 && cell[m] >= 0 && !stay[m]) {
            const int q = atomicAdd(&ws.st->n_mov, 1);
            if (q < ws.N) ws.mov[q] = (uint32_t)cell[m];
        }
    }
    if (!reset) {
        const uint16_t* gene = ws.lay_gene + (int64_t)L * kPlaces;
        for (int j = t; j < D * kBlkGenes; j += kLsThreads) {
            if (DUMP) {
                const int u = gene[j];
                const double v0 = g0[u], v1 = g1[u];
                dl[j] = v1 - v0;
                tl0[j] = v0;
                tl1[j] = v1;
            } else {
                s_lim[j] = ws.lay_lim[(int64_t)L * kPlaces + j];
            }
        }
    }
    if (t < 2) ncnt[t] = ncnt2[t] = 0;
    const int rows = rs ? 4 : 2;
    for (int q = t; q < rows * kPlaces; q += kLsThreads) phist[q / kPlaces][q % kPlaces] = 0;
    __syncthreads();

    // 1. the FP64 sums
    double df[2] = {0.0, 0.0}, s0[2] = {0.0, 0.0}, s1[2] = {0.0, 0.0};
    if (DUMP && !reset) {
        // on the vector ALUs (with the two rows themselves); byte 4p + c of a
        // fragment is place 32 (p >> 1) + 8 g + 4 (p & 1) + c
#pragma unroll 1
        for (int j = 0; j < D; ++j) {
            const uint4 v[2] = {frag(dense, doff, j, 0), frag(dense, doff, j, 1)};
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int place = j * kBlkGenes + 32 * (p >> 1) + 8 * g + 4 * (p & 1) + c;
                    const double dv = dl[place];
#pragma unroll
                    for (int m = 0; m < 2; ++m) {
                        const uint32_t w = p == 0 ? v[m].x : p == 1 ? v[m].y : p == 2 ? v[m].z : v[m].w;
                        const double x = (double)((w >> (8 * c)) & 0xFFu);
                        df[m] = fma(x, dv, df[m]);
                        s0[m] = fma(x, tl0[place], s0[m]);
                        s1[m] = fma(x, tl1[place], s1[m]);
                    }
                }
        }
    }
    if (!DUMP && !reset) {
        // on the matrix cores, exactly: with the digits d_{p,k} of the
        // fixed-point difference v_p (lay_lim), sum_p x_p v_p =
        // sum_k 256^k (sum_p (x_p - 128) d_{p,k} + 128 S_k) over the D chunks,
        // S_k = sum_p d_{p,k} (x - 128 is a signed byte).  Product: digits
        // (A: row k, lane (k, g)) x the lane's own counts (B: column = cell
        // r); lane (r, g) gets the sums of digits k = 4 g .. 4 g + 3 of its
        // cell (rows 7 .. 15 are zero).
        const intx4_t zero = {0, 0, 0, 0};
        intx4_t dacc[2] = {zero, zero};
        const int kr = r < 8 ? r : 7;
        // chunk by chunk, the next chunk's fragments in flight
#pragma unroll 1
        for (int j = 0; j < D; ++j) {
            uint4 n0 = f0, n1 = f1;
            if (j + 1 < D) {
                n0 = frag(dense, doff, j + 1, 0);
                n1 = frag(dense, doff, j + 1, 1);
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const long dig = (long)s_lim[((j * 2 + s) * 8 + kr) * 4 + g];
                dacc[0] = __builtin_amdgcn_mfma_i32_16x16x32_i8(dig, kstep(f0, s) ^ kOffset8, dacc[0], 0, 0, 0);
                dacc[1] = __builtin_amdgcn_mfma_i32_16x16x32_i8(dig, kstep(f1, s) ^ kOffset8, dacc[1], 0, 0, 0);
            }
            f0 = n0;
            f1 = n1;
        }
        const int E = ws.lay_dE[L];
        const int32_t* S = ws.lay_dS + ((int64_t)L * (kLayDmax + 1) + D) * 8;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * g + i;
            const int sk = k < 8 ? S[k] : 0;
#pragma unroll
            for (int m = 0; m < 2; ++m) df[m] += ldexp((double)(dacc[m][i] + 128 * sk), 8 * k - E);
        }
    }
    if (!reset) {
        // the tail: entry tb + g + 4 i of the cell, in entry order
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (!stay[m]) continue;
            int64_t e = tb[m] + g;
            if (!DUMP) {
                if (en0[m]) df[m] = fma((double)(en0[m] >> 16), dt0[m], df[m]);
                e += 4;
            }
            for (; e < te[m]; e += 4) {
                const uint32_t en = ws.lay_tail[e];
                const int u = (int)(en & 0xFFFFu);
                const double x = (double)(en >> 16);
                if (DUMP) {
                    df[m] = fma(x, g1[u] - g0[u], df[m]);
                    s0[m] = fma(x, g0[u], s0[m]);
                    s1[m] = fma(x, g1[u], s1[m]);
                } else {
                    df[m] = fma(x, dfull[u], df[m]);
                }
            }
        }
        // the four lanes of a cell: (own + partner across 16) + (the other pair), the same sum on all four
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            df[m] += __shfl_xor(df[m], 16);
            df[m] += __shfl_xor(df[m], 32);
            if (DUMP) {
                s0[m] += __shfl_xor(s0[m], 16);
                s0[m] += __shfl_xor(s0[m], 32);
                s1[m] += __shfl_xor(s1[m], 16);
                s1[m] += __shfl_xor(s1[m], 32);
            }
        }
    }

    // 2. the draw: lane groups 0 and 1 take the cell of tile 0, groups 2 and
    // 3 that of tile 1; groups 0 and 2 write
    const int md = g >> 1;
    int my_sv = -1, my_cv = 0;
    {
        const bool st = md ? stay[1] : stay[0];
        if (st) {
            const uint32_t i = (uint32_t)(md ? cell[1] : cell[0]);
            double dd = 0.0;
            if (reset) {
                my_sv = (int)(philox(ws.seed, i, 0u, a.step, kResub, 0u).w[0] >> 31);
            } else {
                const double* lw = ws.lay_sw + 4 * (int64_t)L;
                const SubWeights sw{lw[0], lw[1], lw[2], lw[3]};
                my_sv = sub_draw(ws.seed, i, a.step, kGumbelS, sw, md ? ocode[1] : ocode[0],
                                 sub_noise(ws.seed, i, a.step, kGumbelS), md ? df[1] : df[0], &dd);
            }
            if (rs) my_cv = (int)(philox(ws.seed, i, 0u, a.rs_step, kRSplit, 0u).w[0] >> 31);
            if ((g & 1) == 0) {
                a.cs_new[i] = (uint8_t)my_sv;
                if (rs) ws.rbits[i] = (uint8_t)my_cv;
                if (SPLITQ) ws.subdd[i] = reset ? __builtin_nan("") : dd;
                if (a.dbg && K + 2 <= a.dbg_stride) {
                    put_dbg(a.dbg, a.dbg64, (int64_t)i * a.dbg_stride + K,
                            reset || !DUMP ? __builtin_nan("") : (md ? s0[1] : s0[0]));
                    put_dbg(a.dbg, a.dbg64, (int64_t)i * a.dbg_stride + K + 1,
                            reset || !DUMP ? __builtin_nan("") : (md ? s1[1] : s1[0]));
                }
            }
        }
    }
    // both cells' labels on all four lanes of the row
    int sv[2], cv[2];
    {
        const int mine = (my_sv + 1) | (my_cv << 2);
        const int c0 = __shfl(mine, r), c1 = __shfl(mine, 32 + r);
        sv[0] = (c0 & 3) - 1;
        cv[0] = c0 >> 2;
        sv[1] = (c1 & 3) - 1;
        cv[1] = c1 >> 2;
    }
    // the wavefront's cells per statistics row (sub-cluster 0, 1, coin 0, 1)
    uint32_t rc[4];
#pragma unroll
    for (int row = 0; row < 4; ++row) {
        const bool on = row < 2 ? my_sv == row : rs && my_sv >= 0 && my_cv == row - 2;
        rc[row] = (uint32_t)__popcll(__ballot((g & 1) == 0 && on));
    }
    if (lane == 0) {
        if (rc[0]) atomicAdd(&ncnt[0], rc[0]);
        if (rc[1]) atomicAdd(&ncnt[1], rc[1]);
        if (rs && rc[2]) atomicAdd(&ncnt2[0], rc[2]);
        if (rs && rc[3]) atomicAdd(&ncnt2[1], rc[3]);
    }

    // 3. statistics.  Operand byte e of lane group g stands for the
    // wavefront's cell 16 (e >> 2) + 4 g + (e & 3), in both operands of the
    // statistics product (the matrix cores pair the bytes of A and B by lane
    // group and byte alike).  Mask (A): row r of that cell.
    long amask;
    {
        const int code = (sv[0] + 1) | ((sv[1] + 1) << 2) | (cv[0] << 4) | (cv[1] << 5);
        uint64_t mk = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int cd = __shfl(code, 4 * g + i);
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int s = ((cd >> (2 * m)) & 3) - 1, c = (cd >> (4 + m)) & 1;
                const bool on = r < 2 ? s == r : r < 4 && rs && s >= 0 && c == r - 2;
                if (on) mk |= (uint64_t)1 << (8 * (4 * m + i));
            }
        }
        amask = (long)mk;
    }
    // selection (B) of place 16 h + r of a k-step: byte (16 h + r) & 7 of lane group (16 h + r) >> 3
    long sel[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = 16 * h + r;
        sel[h] = g == (q >> 3) ? (long)((uint64_t)1 << (8 * (q & 7))) : 0;
    }
    {
        const int rc128[4] = {128 * (int)rc[0], 128 * (int)rc[1], 128 * (int)rc[2], 128 * (int)rc[3]};
        if (rs) chunk_stats<4>(dense, doff, D, amask, sel, rc128, phist, g, r);
        else chunk_stats<2>(dense, doff, D, amask, sel, rc128, phist, g, r);
    }
    // tail entries of the cells of L, split over the cell's four lanes: a
    // gene among L's first kPlaces places goes to the histogram, any other
    // (rare, and spread over many genes) straight to the statistics
    const uint16_t* rank = ws.lay_rank + (int64_t)L * G;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        if (!stay[m]) continue;
        unsigned long long* srow = ws.ssub + (int64_t)(2 * L + sv[m]) * G;
        unsigned long long* crow = rs ? ws.rssub + (int64_t)(2 * L + cv[m]) * G : nullptr;
        for (int64_t e = tb[m] + g; e < te[m]; e += 4) {
            const bool first = e == tb[m] + g;
            const uint32_t en = first ? en0[m] : ws.lay_tail[e];
            const int p = first ? rk0[m] : rank[en & 0xFFFFu];
            const uint32_t x = en >> 16;
            if (p < kPlaces) {
                atomicAdd(&phist[sv[m]][p], x);
                if (rs) atomicAdd(&phist[2 + cv[m]][p], x);
            } else {
                atomicAdd(&srow[en & 0xFFFFu], (unsigned long long)x);
                if (rs) atomicAdd(&crow[en & 0xFFFFu], (unsigned long long)x);
            }
        }
    }
    __syncthreads();
    {
        uint32_t* part = ws.lay_part + (int64_t)b * ws.lay_pw;
        for (int q = t; q < rows * kPlaces; q += kLsThreads) part[q] = phist[q / kPlaces][q % kPlaces];
    }
    if (t < 2 && ncnt[t]) atomicAdd(&ws.nsub[2 * L + t], (unsigned long long)ncnt[t]);
    if (rs && t < 2 && ncnt2[t]) atomicAdd(&ws.rnsub[2 * L + t], (unsigned long long)ncnt2[t]);
}

// FP64 re-score of a queued cluster decision (eq. 4, third line, with the
// FP64 tables) by the cell's kMovLanes lanes: every lane sums its share of the
// packed row against log theta_k, the shares are combined in a fixed pattern
// that gives all lanes the same value, and the Gumbel-max runs over the K
// clusters in order with FP64 noise.  *near: the relative margin is below
// kNearTie.
__device__ inline int rescore_lanes(const Ws& ws, uint32_t step, uint32_t i, int64_t rb, int64_t re, int lg, int K,
                                    bool* near)
{
    double best = -INFINITY, second = -INFINITY;
    int bk = 0;
    Words w{};
    for (int kk = 0; kk < K; ++kk) {
        const double* lrow = ws.lt64 + (int64_t)kk * ws.G;
        double sk = 0.0;
        for (int64_t p = rb + 4 * lg; p < re; p += 4 * kMovLanes) {
            const uint4 v = *reinterpret_cast<const uint4*>(ws.ent + p);
            const uint32_t en[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t x = en[j] >> 16;
                if (x) sk = fma((double)x, lrow[en[j] & 0xFFFFu], sk);
            }
        }
        for (int o = kMovLanes / 2; o > 0; o >>= 1) sk += __shfl_xor(sk, o, kMovLanes);
        if ((kk & 3) == 0) w = philox(ws.seed, i, (uint32_t)(kk >> 2), step, kGumbelC, 0u);
        const double v = ws.logpi[kk] + sk + (-log(-log(unit23d(w.w[kk & 3]))));
        if (v > best) { second = best; best = v; bk = kk; }
        else if (v > second) second = v;
    }
    *near = K >= 2 && (best - second) / fmax(1.0, fabs(best)) < kNearTie;
    return bk;
}

// The queued cells, each by 8 lanes from the packed matrix: the same FP64 sum
// and draw as the packed-matrix pass, and the statistics with 64-bit atomics.
// An entry flagged kRefineCluster (an uncertain cluster decision of the fused
// pass) is re-scored first.  mb / nmb: this workgroup's index among the nmb
// workgroups that take the queue.
template <bool DUMP, bool SPLITQ>
__device__ void mov_sub(const Ws& ws, const SubArgs& a, int mb, int nmb)
{
    const int n = (int)min((int64_t)ws.st->n_mov, ws.N);
    const int K = ws.st->K;
    const int G = ws.G;
    const bool rs = a.rsplit != 0;
    const int lg = threadIdx.x % kMovLanes;
    const int64_t first = ((int64_t)mb * blockDim.x + threadIdx.x) / kMovLanes;
    const int64_t stride = (int64_t)nmb * blockDim.x / kMovLanes;
    for (int64_t q = first; q < n; q += stride) {
        const uint32_t item = ws.mov[q];
        const uint32_t i = item & ~kRefineCluster;
        const int64_t rb = ws.roff[i], re = ws.roff[i + 1];
        int k;
        if (item & kRefineCluster) {
            bool near;
            k = rescore_lanes(ws, a.step, i, rb, re, lg, K, &near);
            if (lg == 0) {
                a.c_new[i] = k;
                atomicAdd(&ws.st->counters[kCntRefined], 1ull);
                if (near) atomicAdd(&ws.st->counters[kCntNearTie], 1ull);
            }
        } else {
            k = a.c_new[i];
        }
        const bool reset = ws.reset[k] != 0;
        const double* g0 = ws.lt64 + (int64_t)(ws.k_max + 2 * k) * G;
        const double* g1 = g0 + G;
        double df = 0.0, s0 = 0.0, s1 = 0.0;
        if (!reset) {
            for (int64_t p = rb + 4 * lg; p < re; p += 4 * kMovLanes) {
                const uint4 v = *reinterpret_cast<const uint4*>(ws.ent + p);
                const uint32_t en[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t x = en[j] >> 16;
                    if (!x) continue;
                    const int u = (int)(en[j] & 0xFFFFu);
                    df = fma((double)x, g1[u] - g0[u], df);
                    if (DUMP) {
                        s0 = fma((double)x, g0[u], s0);
                        s1 = fma((double)x, g1[u], s1);
                    }
                }
            }
            // sum over the cell's lanes in a fixed order
            for (int o = kMovLanes / 2; o > 0; o >>= 1) {
                df += __shfl_xor(df, o, kMovLanes);
                if (DUMP) {
                    s0 += __shfl_xor(s0, o, kMovLanes);
                    s1 += __shfl_xor(s1, o, kMovLanes);
                }
            }
        }
        int sub;
        double dd = 0.0;
        if (reset) {
            sub = (int)(philox(ws.seed, i, 0u, a.step, kResub, 0u).w[0] >> 31);
        } else {
            const int code = a.c_old[i] == k ? 1 + (a.cs_old[i] & 1) : 0;
            sub = sub_draw(ws.seed, i, a.step, kGumbelS, sub_weights(ws.nsub_prev, k), code,
                           sub_noise(ws.seed, i, a.step, kGumbelS), df, &dd);
        }
        const int coin = rs ? (int)(philox(ws.seed, i, 0u, a.rs_step, kRSplit, 0u).w[0] >> 31) : 0;
        unsigned long long* srow = ws.ssub + (int64_t)(2 * k + sub) * G;
        unsigned long long* crow = rs ? ws.rssub + (int64_t)(2 * k + coin) * G : nullptr;
        for (int64_t p = rb + 4 * lg; p < re; p += 4 * kMovLanes) {
            const uint4 v = *reinterpret_cast<const uint4*>(ws.ent + p);
            const uint32_t en[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const unsigned long long x = en[j] >> 16;
                if (!x) continue;
                atomicAdd(&srow[en[j] & 0xFFFFu], x);
                if (rs) atomicAdd(&crow[en[j] & 0xFFFFu], x);
            }
        }
        if (lg == 0) {
            a.cs_new[i] = (uint8_t)sub;
            atomicAdd(&ws.nsub[2 * k + sub], 1ull);
            if (rs) {
                ws.rbits[i] = (uint8_t)coin;
                atomicAdd(&ws.rnsub[2 * k + coin], 1ull);
            }
            if (SPLITQ) ws.subdd[i] = reset ? __builtin_nan("") : dd;
            if (a.dbg && K + 2 <= a.dbg_stride) {
                put_dbg(a.dbg, a.dbg64, (int64_t)i * a.dbg_stride + K, reset || !DUMP ? __builtin_nan("") : s0);
                put_dbg(a.dbg, a.dbg64, (int64_t)i * a.dbg_stride + K + 1, reset || !DUMP ? __builtin_nan("") : s1);
            }
        }
    }
}

// The blocks' histograms into the statistics.  The blocks of each layout
// cluster L are consecutive, from lay_bbeg[L]; they are cut into spans of
// kRedSpan blocks, lay_sbeg[L] spans before L's first.  A workgroup of kPlaces
// threads sums row r of span x's histograms, place by place, and adds each
// non-zero sum to the statistics of the place's gene with one 64-bit atomic:
// a few per address and span instead of one per count.
__device__ void lay_span(const Ws& ws, int x, int r)
{
    // the span and block offsets of the layout clusters into LDS, then the
    // span's cluster by bisection there
    __shared__ int32_t s_sbeg[kMaxClusters + 1], s_bbeg[kMaxClusters + 1];
    const int KL = ws.st->lay_K;
    const int K = ws.st->K;
    for (int q = threadIdx.x; q <= KL; q += blockDim.x) {
        s_sbeg[q] = ws.lay_sbeg[q];
        s_bbeg[q] = ws.lay_bbeg[q];
    }
    __syncthreads();
    if (x >= s_sbeg[KL]) return;
    int lo = 0, hi = KL;               // s_sbeg[lo] <= x < s_sbeg[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_sbeg[mid] <= x) lo = mid;
        else hi = mid;
    }
    const int L = lo;
    if (L >= K) return;
    const int p = threadIdx.x;
    const int b0 = s_bbeg[L] + (x - s_sbeg[L]) * kRedSpan;
    const int nb = min(s_bbeg[L + 1] - b0, kRedSpan);
    const int64_t pw = ws.lay_pw;
    const uint32_t* in = ws.lay_part + (int64_t)b0 * pw + (int64_t)r * kPlaces + p;
    uint32_t acc = 0;                  // at most kRedSpan x 256 cells x 65535 < 2^32
    // 32 of the span's loads in flight at a time (past its end the last
    // block is read again and not added)
#pragma unroll 1
    for (int i0 = 0; i0 < nb; i0 += 32) {
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            const uint32_t v = in[(int64_t)min(i0 + i, nb - 1) * pw];
            acc += i0 + i < nb ? v : 0u;
        }
    }
    if (!acc) return;
    const int G = ws.G;
    const int u = ws.lay_gene[(int64_t)L * kPlaces + p];
    unsigned long long* dst = r < 2 ? ws.ssub + (int64_t)(2 * L + r) * G + u : ws.rssub + (int64_t)(2 * L + r - 2) * G + u;
    atomicAdd(dst, (unsigned long long)acc);
}

// Both remainders of the pass in one launch (they are independent: both only
// add to the statistics): the first nspan x rows workgroups sum the block
// histograms (span x, row r), the others serve the queue.
template <bool DUMP, bool SPLITQ>
__global__ void __launch_bounds__(kPlaces) k_mov_span(Ws ws, SubArgs a, int nspan, int rows)
{
    const int b = (int)blockIdx.x, ns = nspan * rows;
    if (b < ns) lay_span(ws, b % nspan, b / nspan);
    else mov_sub<DUMP, SPLITQ>(ws, a, b - ns, (int)gridDim.x - ns);
}

using LaySubKernel = void (*)(Ws, SubArgs);

static LaySubKernel lay_sub_kernel(bool dump, bool split_q)
{
    return dump ? (split_q ? k_lay_sub<true, true> : k_lay_sub<true, false>)
                : (split_q ? k_lay_sub<false, true> : k_lay_sub<false, false>);
}

using MovSpanKernel = void (*)(Ws, SubArgs, int, int);

static MovSpanKernel mov_span_kernel(bool dump, bool split_q)
{
    return dump ? (split_q ? k_mov_span<true, true> : k_mov_span<true, false>)
                : (split_q ? k_mov_span<false, true> : k_mov_span<false, false>);
}

// The sub-cluster pass of a split-BF16 sweep: the statistics and counts (and,
// with rsplit, the coin halves') were cleared by the redraw of the same sweep
// (k_redraw_norm), which also emptied the queue of k_mov_span.
void launch_lay_sub(const Ws& ws, const SubArgs& a, hipStream_t s)
{
    const bool dump = a.dbg != nullptr, split_q = ws.subdd != nullptr;
    hipLaunchKernelGGL(lay_sub_kernel(dump, split_q), dim3((unsigned)ws.nblk_cap), dim3(kLsThreads), 0, s, ws, a);
    launch_lay_sub_rest(ws, a, s);
}

void launch_lay_sub_rest(const Ws& ws, const SubArgs& a, hipStream_t s)
{
    const bool dump = a.dbg != nullptr, split_q = ws.subdd != nullptr;
    int64_t mb = (ws.N + kMovGroups - 1) / kMovGroups;
    if (mb > 512) mb = 512;
    const int rows = a.rsplit ? 4 : 2;
    const int nspan = lay_spans(ws.nblk_cap, ws.k_max);
    hipLaunchKernelGGL(mov_span_kernel(dump, split_q), dim3((unsigned)(nspan * rows + mb)), dim3(kPlaces), 0, s, ws, a,
                       nspan, rows);
}

}  // namespace dpmm
