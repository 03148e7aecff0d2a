// laysub.hip -- the sub-cluster draw (Section 2.3, eq. 8) and the integer
// sufficient statistics (step a4) of a split-BF16 sweep, over the
// cluster-sorted copy of the counts (layout.hip) instead of the packed matrix.
//
// A workgroup of 512 threads takes one block of the copy, with layout cluster
// L.  The block's cells whose new label is L (nearly all of them once the
// chain has settled) are drawn here; any other cell of the block goes to a
// queue that k_mov_sub serves from the packed matrix, exactly as the
// packed-matrix pass would.
//   1. Thread (slot, half) loads the half of its cell's dense bytes that it
//      owns, two 16-byte pieces per chunk, all chunks in flight at once, keeps
//      them in registers and forms the FP64 sum of x_u delta_u, with
//      delta_u = log thetabar_{L,1,u} - log thetabar_{L,0,u} staged in LDS in
//      L's gene order; each half adds every other tail entry of the cell, and
//      the halves are added in a fixed order.
//   2. The draw itself (sub_draw, shared with the packed-matrix pass).
//   3. Statistics: chunk by chunk the bytes go to LDS, and the matrix cores
//      form M X, X the chunk's 256 x 64 counts (cells x genes), M the 0/1 rows
//      "cell of L in sub-cluster 0", "... 1" (and "coin 0", "coin 1" of a
//      random split coming next), in BF16 with FP32 accumulation.  Every
//      product and partial sum is an integer below 2^24, so the sums are
//      exact.  The sums go to a per-block LDS histogram over (row, gene),
//      together with the tail entries (a count above 255 is a tail entry too,
//      and those crowd on a cluster's top genes).  Each block writes its whole
//      histogram to lay_part; k_lay_span adds them over spans of consecutive
//      blocks of a cluster and k_lay_reduce adds a cluster's spans into its
//      statistics.  No atomics reach memory: device-scope 64-bit atomics on
//      a few hot addresses from every block serialise.  (Past kLsHistWords
//      histogram words, the sums go to the statistics with atomics instead.)
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4_t;

constexpr int kLsThreads = 2 * kBlkCells;     // two threads per slot
constexpr int kPlaces = kLayDmax * kBlkGenes;  // places of a cluster's gene order in the dense chunks
constexpr int kPartRows = 4;                   // sub-cluster 0, 1, coin 0, 1
constexpr int kMovGroups = 32;                 // cells per workgroup pass of k_mov_sub (8 lanes each)
constexpr int kMovLanes = 8;
constexpr int kRedSpan = kSpanBlocks;

// eight bytes (two words) -> eight BF16 values (exact: each is an integer
// below 256, whose FP32 value has its low 16 bits zero)
__device__ inline bf16x8_t bytes_bf16(uint32_t w0, uint32_t w1)
{
    uint32_t p[4];
    const uint32_t in[2] = {w0, w1};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t v = in[h];
        const uint32_t f0 = __float_as_uint((float)(v & 0xFFu));
        const uint32_t f1 = __float_as_uint((float)((v >> 8) & 0xFFu));
        const uint32_t f2 = __float_as_uint((float)((v >> 16) & 0xFFu));
        const uint32_t f3 = __float_as_uint((float)(v >> 24));
        p[2 * h] = __builtin_amdgcn_perm(f1, f0, 0x07060302u);
        p[2 * h + 1] = __builtin_amdgcn_perm(f3, f2, 0x07060302u);
    }
    bf16x8_t r;
    __builtin_memcpy(&r, p, sizeof(r));
    return r;
}

// The swizzle of a piece's row r in LDS: r ^ (q & 1 | (rt & 1) << 1 | (r >> 3) << 2)
__device__ inline int lane_swizzle(int q, int rt_odd, int r_hi) { return (q & 1) | (rt_odd << 1) | (r_hi << 2); }

template <bool DUMP, bool SPLITQ>
__global__ void __launch_bounds__(kLsThreads) k_lay_sub(Ws ws, SubArgs a)
{
    __shared__ double dl[kPlaces];                         // delta in L's gene order
    __shared__ double tl0[DUMP ? kPlaces : 1], tl1[DUMP ? kPlaces : 1];   // the two rows themselves (dump)
    __shared__ __attribute__((aligned(16))) uint8_t chunk[kDenseChunkBytes];
    __shared__ double hsum[3][2][kBlkCells];               // per-half sums: delta, and rows 0 / 1 (dump)
    __shared__ int8_t s_sub[kBlkCells];                    // sub-label of a cell of L, -1 for any other slot
    __shared__ uint8_t s_coin[kBlkCells];
    __shared__ float psum[2][kPartRows][kBlkGenes];
    __shared__ uint32_t thist[kLsHistWords];               // tail counts per (row, gene)
    __shared__ uint32_t ncnt[2], ncnt2[2];

    const bool rs = a.rsplit != 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) ws.st->rs_live = rs ? 1 : 0;
    const int b = blockIdx.x;
    if (b >= ws.st->lay_nblk) return;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int sl = t & (kBlkCells - 1);
    const int h = t >> 8;                      // which half of the cell's bytes (places 8q .. 8q + 7 of
                                               // both k-steps, q = 2h, 2h + 1)
    const int64_t slot = (int64_t)b * kBlkCells + sl;
    const int L = ws.lay_kc[b];
    const int K = ws.st->K;
    const int G = ws.G;
    const int64_t d0 = ws.lay_doff[b];
    const int D = (int)(ws.lay_doff[b + 1] - d0);
    const int cell = ws.lay_cell[slot];
    const bool stay = cell >= 0 && L < K && a.c_new[cell] == L;
    const bool reset = L < K ? ws.reset[L] != 0 : true;
    const double* g0 = ws.lt64 + (int64_t)(ws.k_max + 2 * (L < K ? L : 0)) * G;
    const double* g1 = g0 + G;

    if (!reset) {
        const uint16_t* gene = ws.lay_gene + (int64_t)L * kPlaces;
        for (int j = t; j < D * kBlkGenes; j += kLsThreads) {
            const int u = gene[j];
            const double v0 = g0[u], v1 = g1[u];
            dl[j] = v1 - v0;
            if (DUMP) {
                tl0[j] = v0;
                tl1[j] = v1;
            }
        }
    }
    if (t < 2) ncnt[t] = ncnt2[t] = 0;
    const int rows = rs ? 4 : 2;
    // LDS offsets of this thread's two pieces of a chunk (swizzled, see below)
    const int rt_me = sl >> 4, r_me = sl & 15;
    const uint32_t w_off0 = (uint32_t)(rt_me * 64 + 16 * (2 * h) + (r_me ^ lane_swizzle(2 * h, rt_me & 1, r_me >> 3))) * 16;
    const uint32_t w_off1 =
        (uint32_t)(rt_me * 64 + 16 * (2 * h + 1) + (r_me ^ lane_swizzle(2 * h + 1, rt_me & 1, r_me >> 3))) * 16;
    const bool lhist = rows * G <= ws.lay_pw;
    if (lhist)
        for (int q = t; q < rows * G; q += kLsThreads) thist[q] = 0;
    if (h == 0 && cell >= 0 && !stay) {
        const int q = atomicAdd(&ws.st->n_mov, 1);
        if (q < ws.N) ws.mov[q] = (uint32_t)cell;
    }
    // the thread's two 16-byte pieces of every chunk
    const uint8_t* dense = ws.lay_dense + d0 * kDenseChunkBytes;       // uniform base
    const uint32_t u0 = (uint32_t)((sl >> 4) * 64 + 32 * h + (sl & 15)) * 16;
    uint4 rv[kLayDmax][2];
#pragma unroll
    for (int j = 0; j < kLayDmax; ++j) {
        if (j < D) {
            rv[j][0] = *reinterpret_cast<const uint4*>(dense + (u0 + (uint32_t)(j * kDenseChunkBytes)));
            rv[j][1] = *reinterpret_cast<const uint4*>(dense + (u0 + (uint32_t)(j * kDenseChunkBytes + 256)));
        } else {
            rv[j][0] = rv[j][1] = make_uint4(0, 0, 0, 0);
        }
    }
    __syncthreads();
    // 1. the FP64 sums; byte 4p + c of a piece is place 32 (p >> 1) + 8 q + 4 (p & 1) + c
    double df = 0.0, s0 = 0.0, s1 = 0.0;
    if (stay && !reset) {
#pragma unroll
        for (int j = 0; j < kLayDmax; ++j) {
            if (j >= D) break;
#pragma unroll
            for (int qq = 0; qq < 2; ++qq) {
                const uint32_t w[4] = {rv[j][qq].x, rv[j][qq].y, rv[j][qq].z, rv[j][qq].w};
                const int q = 2 * h + qq;
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int place = j * kBlkGenes + 32 * (p >> 1) + 8 * q + 4 * (p & 1) + c;
                        const double x = (double)((w[p] >> (8 * c)) & 0xFFu);
                        df = fma(x, dl[place], df);
                        if (DUMP) {
                            s0 = fma(x, tl0[place], s0);
                            s1 = fma(x, tl1[place], s1);
                        }
                    }
            }
        }
        const int64_t tb = ws.lay_toff[slot], te = ws.lay_toff[slot + 1];
        for (int64_t e = tb + h; e < te; e += 2) {
            const uint32_t en = ws.lay_tail[e];
            const int u = (int)(en & 0xFFFFu);
            const double x = (double)(en >> 16);
            df = fma(x, g1[u] - g0[u], df);
            if (DUMP) {
                s0 = fma(x, g0[u], s0);
                s1 = fma(x, g1[u], s1);
            }
        }
    }
    hsum[0][h][sl] = df;
    if (DUMP) {
        hsum[1][h][sl] = s0;
        hsum[2][h][sl] = s1;
    }
    __syncthreads();
    // 2. the draw
    if (h == 0) {
        int sv = -1, cv = 0;
        if (stay) {
            const uint32_t i = (uint32_t)cell;
            double dd = 0.0;
            if (reset) {
                sv = (int)(philox(ws.seed, i, 0u, a.step, kResub, 0u).w[0] >> 31);
            } else {
                const int code = a.c_old[cell] == L ? 1 + (a.cs_old[cell] & 1) : 0;
                sv = sub_draw(ws.seed, i, a.step, kGumbelS, sub_weights(ws.nsub_prev, L), code,
                              sub_noise(ws.seed, i, a.step, kGumbelS), hsum[0][0][sl] + hsum[0][1][sl], &dd);
            }
            a.cs_new[cell] = (uint8_t)sv;
            atomicAdd(&ncnt[sv], 1u);
            if (rs) {
                cv = (int)(philox(ws.seed, i, 0u, a.rs_step, kRSplit, 0u).w[0] >> 31);
                ws.rbits[cell] = (uint8_t)cv;
                atomicAdd(&ncnt2[cv], 1u);
            }
            if (SPLITQ) ws.lpsub[cell] = reset ? 0.0 : sub_logp(dd, sv);
            if (a.dbg && K + 2 <= a.dbg_stride) {
                put_dbg(a.dbg, a.dbg64, (int64_t)cell * a.dbg_stride + K,
                        reset || !DUMP ? __builtin_nan("") : hsum[1][0][sl] + hsum[1][1][sl]);
                put_dbg(a.dbg, a.dbg64, (int64_t)cell * a.dbg_stride + K + 1,
                        reset || !DUMP ? __builtin_nan("") : hsum[2][0][sl] + hsum[2][1][sl]);
            }
        }
        s_sub[sl] = (int8_t)sv;
        s_coin[sl] = (uint8_t)cv;
    }
    __syncthreads();
    // tail entries of the cells of L: every other one per half
    if (stay) {
        const int sv = s_sub[sl], cv = s_coin[sl];
        const int64_t tb = ws.lay_toff[slot], te = ws.lay_toff[slot + 1];
        if (lhist) {
            uint32_t* hs = thist + sv * G;
            uint32_t* hc = thist + (2 + cv) * G;
            for (int64_t e = tb + h; e < te; e += 2) {
                const uint32_t en = ws.lay_tail[e];
                atomicAdd(&hs[en & 0xFFFFu], en >> 16);
                if (rs) atomicAdd(&hc[en & 0xFFFFu], en >> 16);
            }
        } else {
            unsigned long long* srow = ws.ssub + (int64_t)(2 * L + sv) * G;
            unsigned long long* crow = rs ? ws.rssub + (int64_t)(2 * L + cv) * G : nullptr;
            for (int64_t e = tb + h; e < te; e += 2) {
                const uint32_t en = ws.lay_tail[e];
                const unsigned long long x = en >> 16;
                atomicAdd(&srow[en & 0xFFFFu], x);
                if (rs) atomicAdd(&crow[en & 0xFFFFu], x);
            }
        }
    }
    // 3. dense statistics on the matrix cores.  Wavefront w takes the genes of
    // column tile w & 3 against cells 128 (w >> 2) .. + 127 (four k-steps of
    // 32); the mask rows (A operand: lane l holds row l % 16 for cells
    // 8 (l / 16) .. + 7 of a k-step) are fixed for the block.
    const int nt = wave & 3, kh = wave >> 2;
    bf16x8_t am[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        uint16_t m16[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int c = 128 * kh + 32 * ks + 8 * (lane >> 4) + e;
            const int m = lane & 15;
            const int sv = s_sub[c];
            bool on = false;
            if (m < 2) on = sv == m;
            else if (m < 4) on = rs && sv >= 0 && (int)s_coin[c] == m - 2;
            m16[e] = on ? (uint16_t)0x3F80u : (uint16_t)0u;   // BF16 1.0 or 0
        }
        __builtin_memcpy(&am[ks], m16, sizeof(m16));
    }
    // B operand: lane l holds gene 16 nt + l % 16 for cells 8 (l / 16) .. + 7
    // of a k-step.  In LDS the chunk keeps its fragment order (16-byte piece
    // 64 rt + 16 q + r: cell 16 rt + r, places 8 q .. + 7 and 32 + 8 q .. + 7)
    // except that r is stored as r ^ swz(q, rt, r >> 3): the eight pieces a
    // lane reads, and the lanes of one read, then fall on distinct banks.
    const int g = 16 * nt + (lane & 15);
    const int qg = (g >> 3) & 3;
    const uint32_t gbyte = (uint32_t)(16 * qg) * 16 + (uint32_t)(g >> 5) * 8 + (uint32_t)(g & 7);
    const int swz_l = lane_swizzle(qg, lane >> 5, (lane >> 4) & 1);   // (rt & 1, r >> 3 of this lane's cells)
    const uint16_t* gene_of = ws.lay_gene + (int64_t)L * kPlaces;
#pragma unroll 1
    for (int j = 0; j < D; ++j) {
        __syncthreads();                       // the previous chunk's readers are done
        *reinterpret_cast<uint4*>(chunk + w_off0) = rv[0][0];
        *reinterpret_cast<uint4*>(chunk + w_off1) = rv[0][1];
        // rotate the chunks so that the one just stored is dropped (constant indices only)
#pragma unroll
        for (int jj = 0; jj + 1 < kLayDmax; ++jj) {
            rv[jj][0] = rv[jj + 1][0];
            rv[jj][1] = rv[jj + 1][1];
        }
        __syncthreads();
        floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int c0 = 128 * kh + 32 * ks + 8 * (lane >> 4);
            const uint8_t* src = chunk + (uint32_t)((c0 >> 4) * 64 + (c0 & 15)) * 16 + gbyte;
            uint32_t w0 = 0, w1 = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                w0 |= (uint32_t)src[16 * (e ^ swz_l)] << (8 * e);
                w1 |= (uint32_t)src[16 * ((e + 4) ^ swz_l)] << (8 * e);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[ks], bytes_bf16(w0, w1), acc, 0, 0, 0);
        }
        // rows 0 .. 3 of the tile are in lanes 0 .. 15, row i in acc[i]
        if (lane < 16)
#pragma unroll
            for (int i = 0; i < kPartRows; ++i) psum[kh][i][16 * nt + lane] = acc[i];
        __syncthreads();
        if (t < rows * kBlkGenes) {
            const int r = t / kBlkGenes, gg = t % kBlkGenes;
            const uint32_t v = (uint32_t)(psum[0][r][gg] + psum[1][r][gg]);
            if (v) {
                const int u = gene_of[j * kBlkGenes + gg];
                if (lhist) {
                    atomicAdd(&thist[r * G + u], v);
                } else {
                    unsigned long long* dst = r < 2 ? ws.ssub + (int64_t)(2 * L + r) * G + u
                                                    : ws.rssub + (int64_t)(2 * L + r - 2) * G + u;
                    atomicAdd(dst, (unsigned long long)v);
                }
            }
        }
    }
    if (lhist) {
        __syncthreads();
        uint32_t* part = ws.lay_part + (int64_t)b * ws.lay_pw;
        for (int q = t; q < rows * G; q += kLsThreads) part[q] = thist[q];
    }
    if (t < 2 && ncnt[t]) atomicAdd(&ws.nsub[2 * L + t], (unsigned long long)ncnt[t]);
    if (rs && t < 2 && ncnt2[t]) atomicAdd(&ws.rnsub[2 * L + t], (unsigned long long)ncnt2[t]);
}

// The queued cells, each by 8 lanes from the packed matrix: the same FP64 sum
// and draw as the packed-matrix pass, and the statistics with 64-bit atomics.
template <bool DUMP, bool SPLITQ>
__global__ void __launch_bounds__(256) k_mov_sub(Ws ws, SubArgs a)
{
    const int n = (int)min((int64_t)ws.st->n_mov, ws.N);
    const int K = ws.st->K;
    const int G = ws.G;
    const bool rs = a.rsplit != 0;
    const int lg = threadIdx.x % kMovLanes;
    const int64_t first = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kMovLanes;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / kMovLanes;
    for (int64_t q = first; q < n; q += stride) {
        const uint32_t i = ws.mov[q];
        const int k = a.c_new[i];
        const bool reset = ws.reset[k] != 0;
        const double* g0 = ws.lt64 + (int64_t)(ws.k_max + 2 * k) * G;
        const double* g1 = g0 + G;
        const int64_t rb = ws.roff[i], re = ws.roff[i + 1];
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
            if (SPLITQ) ws.lpsub[i] = reset ? 0.0 : sub_logp(dd, sub);
            if (a.dbg && K + 2 <= a.dbg_stride) {
                put_dbg(a.dbg, a.dbg64, (int64_t)i * a.dbg_stride + K, reset || !DUMP ? __builtin_nan("") : s0);
                put_dbg(a.dbg, a.dbg64, (int64_t)i * a.dbg_stride + K + 1, reset || !DUMP ? __builtin_nan("") : s1);
            }
        }
    }
}

// The blocks' histograms into the statistics, in two passes without atomics.
// The blocks of each layout cluster L are consecutive, from lay_bbeg[L]; they
// are cut into spans of kRedSpan blocks, lay_sbeg[L] spans before L's first.
// k_lay_span: workgroup x sums span x's histograms into span_part[x];
// k_lay_reduce: entry (r, u) of cluster L, the sum over L's spans, added to
// the statistics by the one thread that owns it.
__global__ void __launch_bounds__(kLsThreads) k_lay_span(Ws ws, int rows)
{
    const int KL = ws.st->lay_K;
    const int x = blockIdx.x;
    if (x >= ws.lay_sbeg[KL]) return;
    int lo = 0, hi = KL;               // lay_sbeg[lo] <= x < lay_sbeg[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ws.lay_sbeg[mid] <= x) lo = mid;
        else hi = mid;
    }
    const int L = lo;
    const int b0 = ws.lay_bbeg[L] + (x - ws.lay_sbeg[L]) * kRedSpan;
    const int nb = min(ws.lay_bbeg[L + 1] - b0, kRedSpan);
    const int64_t pw = ws.lay_pw;
    const uint32_t* in = ws.lay_part + (int64_t)b0 * pw;
    uint32_t* out = ws.span_part + (int64_t)x * pw;
    const int n = rows * ws.G;
    for (int q = threadIdx.x; q < n; q += kLsThreads) {
        uint32_t acc = 0;              // at most kRedSpan x 256 cells x 65535 < 2^32
#pragma unroll 8
        for (int i = 0; i < nb; ++i) acc += in[(int64_t)i * pw + q];
        out[q] = acc;
    }
}

__global__ void __launch_bounds__(256) k_lay_reduce(Ws ws, int rows)
{
    const int L = blockIdx.y;
    if (L >= ws.st->lay_K || L >= ws.st->K) return;
    const int G = ws.G;
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= rows * G) return;
    const int x0 = ws.lay_sbeg[L], x1 = ws.lay_sbeg[L + 1];
    const int64_t pw = ws.lay_pw;
    unsigned long long acc = 0;
#pragma unroll 4
    for (int x = x0; x < x1; ++x) acc += ws.span_part[(int64_t)x * pw + q];
    if (!acc) return;
    const int r = q / G, u = q - r * G;
    if (r < 2) ws.ssub[(int64_t)(2 * L + r) * G + u] += acc;
    else ws.rssub[(int64_t)(2 * L + r - 2) * G + u] += acc;
}

using LaySubKernel = void (*)(Ws, SubArgs);

static LaySubKernel lay_sub_kernel(bool dump, bool split_q)
{
    return dump ? (split_q ? k_lay_sub<true, true> : k_lay_sub<true, false>)
                : (split_q ? k_lay_sub<false, true> : k_lay_sub<false, false>);
}

static LaySubKernel mov_sub_kernel(bool dump, bool split_q)
{
    return dump ? (split_q ? k_mov_sub<true, true> : k_mov_sub<true, false>)
                : (split_q ? k_mov_sub<false, true> : k_mov_sub<false, false>);
}

// The sub-cluster pass of a split-BF16 sweep: the statistics and counts were
// cleared by the redraw of the same sweep (k_redraw_norm), which also emptied
// the queue of k_mov_sub.
void launch_lay_sub(const Ws& ws, const SubArgs& a, hipStream_t s)
{
    if (a.rsplit) {
        launch_zero(ws.rssub, sizeof(unsigned long long) * 2 * (size_t)ws.k_max * (size_t)ws.G, s);
        launch_zero(ws.rnsub, sizeof(unsigned long long) * 2 * (size_t)ws.k_max, s);
    }
    const bool dump = a.dbg != nullptr, split_q = ws.lpsub != nullptr;
    hipLaunchKernelGGL(lay_sub_kernel(dump, split_q), dim3((unsigned)ws.nblk_cap), dim3(kLsThreads), 0, s, ws, a);
    int64_t mb = (ws.N + kMovGroups - 1) / kMovGroups;
    if (mb > 1024) mb = 1024;
    hipLaunchKernelGGL(mov_sub_kernel(dump, split_q), dim3((unsigned)mb), dim3(kMovGroups * kMovLanes), 0, s, ws, a);
    const int rows = a.rsplit ? 4 : 2;
    if (rows * ws.G <= ws.lay_pw) {
        hipLaunchKernelGGL(k_lay_span, dim3((unsigned)lay_spans(ws.nblk_cap, ws.k_max)), dim3(kLsThreads), 0, s, ws,
                           rows);
        hipLaunchKernelGGL(k_lay_reduce, dim3((unsigned)((rows * ws.G + 255) / 256), (unsigned)ws.k_max), dim3(256), 0,
                           s, ws, rows);
    }
}

}  // namespace dpmm
