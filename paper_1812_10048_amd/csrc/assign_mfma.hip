// assign_mfma.hip -- the cluster draw (eq. 4, third line) with the cluster
// log-likelihoods S_ik = sum_u x_i^u log theta_{k,u} (eq. 26) on the matrix
// cores, over the cluster-sorted copy of the counts built in layout.hip.
//
// A workgroup of 8 wavefronts owns one block of kBlkCells cells of one layout
// cluster L; wavefront w owns slots 32w .. 32w + 31 (2 row tiles of 16).  The
// block's first D_b chunks of kBlkGenes genes (in L's gene order) are dense
// counts, one byte each, stored in the order of the MFMA A fragments, so each
// lane reads its two k-steps of a row tile with one 16-byte load and widens
// the bytes to BF16 (exact: counts <= 255).  log theta = hi + lo in BF16 comes
// from the same gene order (layout.hip, k_lay_btab).  The chunks go in groups
// of up to kStageChunks: each lane issues the loads of all its A fragments of
// the group while the workgroup stages the group's hi/lo rows in LDS, then
// each wavefront issues
// 2 k-steps x 2 row tiles x NT column tiles x 2 (hi, lo)
// v_mfma_f32_16x16x32_bf16 per chunk.  Every other entry of a cell (a gene
// past the dense chunks, or a count above 255) is in the cell's tail list and
// adds x * fp32(log theta) on the vector ALUs.  Two threads per cell then
// take the Gumbel-max over half of the K scores each, and merge their two
// best; a decision within the certified rounding bound of its two best
// scores (or within the near-tie margin) is queued for the FP64 re-score.
//
// Rounding bound of a score S (all terms x log theta <= 0):
//   * representation: |log theta - hi - lo| <= 2^-17 |log theta| (dense
//     part), |log theta - fp32(log theta)| <= 2^-24 |log theta| (tail);
//   * products: a count <= 255 times a BF16 value is exact in FP32; a tail
//     product is rounded once;
//   * sums: however the matrix core orders and rounds the additions inside
//     and across v_mfma_f32_16x16x32_bf16, each addition of two non-zero FP32
//     values is taken to err by at most one unit in the last place (2^-23
//     relative, which covers round-to-nearest and truncation), adding a zero
//     is exact, and every partial sum is bounded by the sum of the magnitudes
//     of its terms; a cell with n non-zero counts has at most 2n dense terms
//     (hi and lo) and n tail terms, so at most 2n + 8 inexact additions
//     including the tail, log pi and the Gumbel noise;
//   * the FP32 Gumbel noise is within 1e-5 of the FP64 noise.
// bound = (2^-17 + (2n + 8) 2^-23) 1.01 (|S| + |log pi| + 20) + 1e-5.
#include "dpmm_common.hpp"
#include "kernels.hpp"
#include "laystats.hpp"

namespace dpmm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4_t;

constexpr int kMfmaThreads = 2 * kBlkCells;   // 512: two threads per block slot
constexpr int kStageChunks = 3;               // dense chunks whose B rows are staged in LDS at a time
constexpr int kTailStage = 2048;              // tail entries of a block staged in LDS (more: read from memory)
constexpr int kTailBatch = 2;                 // tail entries whose table rows a thread has in flight together
constexpr int kRowB = kBlkGenes + 8;          // BF16 elements per staged B row (padded against bank conflicts)

__host__ __device__ constexpr size_t mfma_lds_bytes(int nt)
{
    // hi/lo B rows of kStageChunks chunks, or the FP32 score tile reusing them
    return (size_t)kStageChunks * 2 * 16 * nt * kRowB * 2 > (size_t)kBlkCells * (16 * nt + 1) * 4
               ? (size_t)kStageChunks * 2 * 16 * nt * kRowB * 2
               : (size_t)kBlkCells * (16 * nt + 1) * 4;
}

__device__ inline float gumbel32(uint32_t w) { return -logf(-logf(unit23f(w))); }
// bounds of -log(-log(u)) over the u23 values, (0.5 .. 2^23 - 0.5) 2^-23:
// -2.8122 and 16.6355, widened for the FP32 logarithms
constexpr float kGumbelLo = -2.82f;
constexpr float kGumbelHi = 16.65f;

__device__ inline float bf16_bound(float acc, float lp, int nnz)
{
    return (0x1p-17f + (float)(2 * nnz + 8) * 0x1p-23f) * 1.01f * (fabsf(acc) + fabsf(lp) + 20.0f) + 1e-5f;
}

// four count bytes -> four BF16 values, two per 32-bit word (the FP32 value of
// a byte has its low 16 bits zero, so its high half is the exact BF16)
__device__ inline void widen4(uint32_t v, uint32_t& lo2, uint32_t& hi2)
{
    // (byte -> float is one v_cvt_f32_ubyteN each)
    const uint32_t f0 = __float_as_uint((float)(v & 0xFFu));
    const uint32_t f1 = __float_as_uint((float)((v >> 8) & 0xFFu));
    const uint32_t f2 = __float_as_uint((float)((v >> 16) & 0xFFu));
    const uint32_t f3 = __float_as_uint((float)(v >> 24));
    lo2 = __builtin_amdgcn_perm(f1, f0, 0x07060302u);
    hi2 = __builtin_amdgcn_perm(f3, f2, 0x07060302u);
}

// eight count bytes (two words) -> one A fragment of 8 BF16
__device__ inline bf16x8_t widen8(uint32_t w0, uint32_t w1)
{
    uint32_t p[4];
    widen4(w0, p[0], p[1]);
    widen4(w1, p[2], p[3]);
    bf16x8_t r;
    __builtin_memcpy(&r, p, sizeof(r));
    return r;
}

// the same for high-plane bytes, times 256 (exact: 8 significant bits)
__device__ inline bf16x8_t widen8_x256(uint32_t w0, uint32_t w1)
{
    uint32_t p[4];
    const uint32_t w[2] = {w0, w1};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t f0 = __float_as_uint((float)(w[h] & 0xFFu) * 256.0f);
        const uint32_t f1 = __float_as_uint((float)((w[h] >> 8) & 0xFFu) * 256.0f);
        const uint32_t f2 = __float_as_uint((float)((w[h] >> 16) & 0xFFu) * 256.0f);
        const uint32_t f3 = __float_as_uint((float)(w[h] >> 24) * 256.0f);
        p[2 * h] = __builtin_amdgcn_perm(f1, f0, 0x07060302u);
        p[2 * h + 1] = __builtin_amdgcn_perm(f3, f2, 0x07060302u);
    }
    bf16x8_t r;
    __builtin_memcpy(&r, p, sizeof(r));
    return r;
}

// The best two Gumbel-perturbed scores seen: value, score and log pi of each.
struct Top2 {
    float t1, t2, a1, a2, p1, p2;
    int k1;
    __device__ inline void init()
    {
        t1 = t2 = -INFINITY;
        a1 = a2 = p1 = p2 = 0.f;
        k1 = 0;
    }
    __device__ inline void add(float v, float s, float lp, int k)
    {
        if (v > t1) {
            t2 = t1; a2 = a1; p2 = p1;
            t1 = v; a1 = s; p1 = lp; k1 = k;
        } else if (v > t2) {
            t2 = v; a2 = s; p2 = lp;
        }
    }
};

// (4 wavefronts per SIMD hold NT <= 3 without spilling; NT = 4 takes the registers of 2)
template <int NT, bool SUB>
__global__ void __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(NT >= 4 ? 2 : 4)))
k_assign_bf16(Ws ws, AssignArgs a, SubArgs sa)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    uint16_t* bst = reinterpret_cast<uint16_t*>(lds);                 // [chunk][hi, lo][16 NT][kRowB]
    float* sc = reinterpret_cast<float*>(lds);                         // epilogue alias [256][16 NT + 1]
    __shared__ float x_t1[kBlkCells], x_t2[kBlkCells], x_a1[kBlkCells], x_a2[kBlkCells], x_p1[kBlkCells],
        x_p2[kBlkCells];
    __shared__ int x_k1[kBlkCells];
    __shared__ float x_d[2][kBlkCells];        // each half's best score + log pi
    __shared__ uint32_t t_ent[kTailStage];     // the block's tail entries
    __shared__ float s_lp[kMaxClusters];       // log pi in FP32
    __shared__ int8_t s_sub[SUB ? kBlkCells : 1];             // fused sub-cluster pass: each slot's sub-label
    __shared__ uint8_t s_coin[SUB ? kBlkCells : 1];           // (-1: not drawn here) and coin
    __shared__ uint32_t s_ncnt[4];
    __shared__ uint8_t s_hcnt[kBlkCells];      // each slot's high-plane tail entries
    __shared__ uint32_t s_tbo[kBlkCells], s_teo[kBlkCells];   // each slot's tail, from the block's first
    __shared__ double s_dfd[SUB ? kBlkCells : 1];
    __shared__ int s_old[SUB ? kBlkCells : 1];               // (old cluster << 1) | old sub-label
    constexpr int SS = 16 * NT + 1;
    constexpr int NCOL = 16 * NT;
    constexpr int HALF = NCOL / 2;             // clusters per thread of a slot's pair (multiple of 8)

    if (SUB && blockIdx.x == 0 && threadIdx.x == 0) ws.st->rs_live = sa.rsplit ? 1 : 0;
    // XCD-aware order: workgroups are dealt to the 8 XCDs in turn (workgroup i
    // to XCD i % 8), and each XCD takes one contiguous range of the live
    // blocks, so the blocks of a cluster, which share its tables, run on one
    // XCD and its L2 (a bijection of [0, nb))
    const int nb = ws.st->lay_nblk;
    if ((int)blockIdx.x >= nb) return;
    const int b = [&] {
        const int x = blockIdx.x & 7, i = blockIdx.x >> 3, q = nb >> 3, r = nb & 7;
        return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
    }();
    const int K = ws.st->K;
    // with the fused sub-cluster pass the digit columns K .. K + kSubDigits - 1
    // of the hi/lo tables are scored too
    const int KC = SUB ? K + kSubDigits : K;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;                   // 8 wavefronts, 32 slots (two row tiles) each
    const int sl = t & (kBlkCells - 1);        // the slot of this thread in the epilogue
    const int half = t >> 8;                   // which half of a column group it takes
    const int64_t slot = (int64_t)b * kBlkCells + sl;
    const int cell = ws.lay_cell[slot];
    // (fused pass) the cell's old labels, needed by its draw at the end, kept in LDS
    if (SUB && half == 0) s_old[sl] = cell >= 0 ? (sa.c_old[cell] << 1) | (sa.cs_old[cell] & 1) : 0;
    const int L = ws.lay_kc[b];
    const int64_t d0 = ws.lay_doff[b];
    const int HP = ws.lay_bh[b];               // a high plane after the D dense chunks
    const int D = (int)(ws.lay_doff[b + 1] - d0) - HP;
    // this lane's 16 bytes of row tile 2w + m of chunk j: + j chunk + m 1 KiB
    const uint8_t* dense = ws.lay_dense + d0 * kDenseChunkBytes;   // uniform base
    const uint32_t doff = (uint32_t)((wave * 2) * 64 + lane) * 16;
    // the slot's tail [tb, te) is kept in LDS as offsets from the block's
    // (registers are short across the chunk loop)
    const int64_t tbase = ws.lay_toff[(int64_t)b * kBlkCells];
    if (half == 0) {
        s_tbo[sl] = (uint32_t)(ws.lay_toff[slot] - tbase);
        s_teo[sl] = (uint32_t)(ws.lay_toff[slot + 1] - tbase);
    }
    // the cluster scores take the tail up to the high-plane entries (the
    // plane's MFMA covers those; their count kept in LDS until the tail walk);
    // the draw and the statistics take all of it
    if (half == 0) s_hcnt[sl] = ws.lay_hcnt[slot];
    // the block's tail entries are contiguous: one coalesced copy into LDS,
    // read after the first barrier below
    const int64_t tcount = ws.lay_toff[(int64_t)(b + 1) * kBlkCells] - tbase;
    const bool staged = tcount <= kTailStage;
    if (staged)
        for (int i = t; i < (int)tcount; i += kMfmaThreads) t_ent[i] = ws.lay_tail[tbase + i];
    // (both read after the first barrier below)
    for (int k = t; k < K; k += kMfmaThreads) s_lp[k] = (float)ws.logpi[k];
    constexpr int R = kLayDmax * kBlkGenes;

    Top2 top;
    top.init();
    // (fused pass: the cell's digit sums combined in FP64, s_dfd[sl], kept in
    // LDS across the column groups)
    if (SUB && half == 0) s_dfd[sl] = 0.0;
    const int dE = SUB && L < K ? ws.lay_dE[L] : 0;
    if (SUB && t < 4) s_ncnt[t] = 0;

    for (int kb = 0; kb < KC; kb += NCOL) {
        floatx4_t acc[2][NT];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[m][n] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
        for (int g0 = 0; g0 < kLayDmax; g0 += kStageChunks) {
            if (g0 >= D) break;                // uniform across the workgroup
            const int gn = min(kStageChunks, D - g0);
            // the group's A fragments in flight while its B rows are staged
            uint4 av[kStageChunks][2];
#pragma unroll
            for (int jj = 0; jj < kStageChunks; ++jj)
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    av[jj][m] = jj < gn ? *reinterpret_cast<const uint4*>(dense + (doff + (uint32_t)((g0 + jj) * kDenseChunkBytes + m * 1024)))
                                        : make_uint4(0, 0, 0, 0);
            __syncthreads();                   // the previous readers of the LDS are done
            {
                // B rows: gn chunks x (hi, lo) x NCOL columns x 8 pieces of 16 bytes
                const int items = gn * 2 * NCOL * (kBlkGenes / 8);
                const uint16_t* hi = ws.lay_bhi + ((int64_t)L * ws.lay_cols + kb) * R + g0 * kBlkGenes;
                const uint16_t* lo = ws.lay_blo + ((int64_t)L * ws.lay_cols + kb) * R + g0 * kBlkGenes;
                for (int q = t; q < items; q += kMfmaThreads) {
                    const int piece = q & 7;
                    const int col = (q >> 3) % NCOL;
                    const int rest = (q >> 3) / NCOL;      // jj * 2 + tbl
                    const int tbl = rest & 1, jj = rest >> 1;
                    const uint16_t* src = (tbl ? lo : hi) + (int64_t)col * R + jj * kBlkGenes + piece * 8;
                    *reinterpret_cast<uint4*>(bst + (rest * NCOL + col) * kRowB + piece * 8) =
                        *reinterpret_cast<const uint4*>(src);
                }
            }
            __syncthreads();
#pragma unroll
            for (int jj = 0; jj < kStageChunks; ++jj) {
                if (jj >= gn) break;
                bf16x8_t af[2][2];
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    af[m][0] = widen8(av[jj][m].x, av[jj][m].y);
                    af[m][1] = widen8(av[jj][m].z, av[jj][m].w);
                }
                const uint16_t* bh = bst + (2 * jj) * NCOL * kRowB;
                const uint16_t* bl = bst + (2 * jj + 1) * NCOL * kRowB;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int col = 32 * s + 8 * (lane >> 4);
#pragma unroll
                    for (int n = 0; n < NT; ++n) {
                        const bf16x8_t vh = *reinterpret_cast<const bf16x8_t*>(bh + (16 * n + (lane & 15)) * kRowB + col);
                        const bf16x8_t vl = *reinterpret_cast<const bf16x8_t*>(bl + (16 * n + (lane & 15)) * kRowB + col);
#pragma unroll
                        for (int m = 0; m < 2; ++m) {
                            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[m][s], vh, acc[m][n], 0, 0, 0);
                            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[m][s], vl, acc[m][n], 0, 0, 0);
                        }
                    }
                }
            }
            if (g0 == 0 && HP) {
                // the high plane (256 x the high bytes of the counts above 255
                // on chunk 0's first kPlaneGenes places, one k-step, 8 bytes
                // per lane) against chunk 0's B rows, still staged; the digit
                // columns see zeros (their sums stay exact integers of the low
                // bytes; the high part of the score difference comes with the
                // cell's tail entries).  One row tile at a time.
                const uint16_t* bh = bst;
                const uint16_t* bl = bst + NCOL * kRowB;
                const bf16x8_t zero8 = {};
                const int col = 8 * (lane >> 4);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const uint2 hv = *reinterpret_cast<const uint2*>(dense + ((doff >> 1) + (uint32_t)(D * kDenseChunkBytes + m * 512)));
                    const bf16x8_t hf = widen8_x256(hv.x, hv.y);
#pragma unroll
                    for (int n = 0; n < NT; ++n) {
                        const int c = kb + 16 * n + (lane & 15);
                        const bool digit = c >= K && c < K + kSubDigits;
                        const bf16x8_t vh = digit ? zero8 : *reinterpret_cast<const bf16x8_t*>(bh + (16 * n + (lane & 15)) * kRowB + col);
                        const bf16x8_t vl = digit ? zero8 : *reinterpret_cast<const bf16x8_t*>(bl + (16 * n + (lane & 15)) * kRowB + col);
                        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hf, vh, acc[m][n], 0, 0, 0);
                        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hf, vl, acc[m][n], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
        // scores through LDS: lane l holds, for row tile m and column tile n,
        // slots 32w + 16m + 4(l/16) + q (q < 4) against cluster kb + 16n + l%16
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    sc[(32 * wave + 16 * m + 4 * (lane >> 4) + q) * SS + 16 * n + (lane & 15)] = acc[m][n][q];
        __syncthreads();
        if (SUB && half == 0) {
            // the digit sums of this group's columns (exact integers in FP32;
            // read before the tail adds to them)
#pragma unroll
            for (int k = 0; k < kSubDigits; ++k) {
                const int col = K + k - kb;
                if (col >= 0 && col < NCOL) s_dfd[sl] += ldexp((double)sc[sl * SS + col], 8 * k - dE);
            }
        }
        if (cell >= 0) {
            // this thread's half of the column group: HALF clusters from kh
            const int kh = kb + half * HALF;
            // the cell's tail entries in FP32 against the gene-major table,
            // added in entry order to this thread's own columns of the score
            // row, two entries' table rows in flight at a time
            float* srow = sc + sl * SS + half * HALF;
            const int64_t tb = tbase + s_tbo[sl];
            const int64_t te = tbase + s_teo[sl] - s_hcnt[sl];     // (without the high-plane entries)
            if (te > tb) {
                float ta[HALF];
#pragma unroll
                for (int k = 0; k < HALF; ++k) ta[k] = srow[k];
                const float* lcb = ws.lc32 + kh;
                // kTailBatch entries' table rows in flight at a time; past the
                // end the last entry is read again and counts zero (adding
                // 0 x a finite log theta leaves the sum unchanged)
#pragma unroll 1
                for (int64_t e = tb; e < te; e += kTailBatch) {
                    uint32_t nn[kTailBatch];
                    float xs[kTailBatch];
#pragma unroll
                    for (int i = 0; i < kTailBatch; ++i) {
                        const int64_t ei = e + i < te ? e + i : te - 1;
                        nn[i] = staged ? t_ent[ei - tbase] : ws.lay_tail[ei];
                        xs[i] = e + i < te ? (float)(nn[i] >> 16) : 0.0f;
                    }
                    float4 v[kTailBatch][HALF / 4];
#pragma unroll
                    for (int i = 0; i < kTailBatch; ++i) {
                        const float4* row = reinterpret_cast<const float4*>(lcb + (int64_t)(nn[i] & 0xFFFFu) * ws.kpad);
#pragma unroll
                        for (int k4 = 0; k4 < HALF / 4; ++k4) v[i][k4] = row[k4];
                    }
#pragma unroll
                    for (int i = 0; i < kTailBatch; ++i)
#pragma unroll
                        for (int k4 = 0; k4 < HALF / 4; ++k4) {
                            ta[4 * k4 + 0] = fmaf(xs[i], v[i][k4].x, ta[4 * k4 + 0]);
                            ta[4 * k4 + 1] = fmaf(xs[i], v[i][k4].y, ta[4 * k4 + 1]);
                            ta[4 * k4 + 2] = fmaf(xs[i], v[i][k4].z, ta[4 * k4 + 2]);
                            ta[4 * k4 + 3] = fmaf(xs[i], v[i][k4].w, ta[4 * k4 + 3]);
                        }
                }
#pragma unroll
                for (int k = 0; k < HALF; ++k) srow[k] = ta[k];
            }
            // Gumbel pruning.  Scores and log pi are <= 0, so a cluster's
            // rounding bound grows with |score + log pi|.  The noise of a
            // draw lies in [kGumbelLo, kGumbelHi]; a cluster whose score plus
            // log pi is below the group's best by more than that width plus
            // both clusters' rounding bounds and the refinement margins can
            // neither win nor be the runner-up of an uncertified decision, in
            // FP32 or in exact arithmetic, so its noise is not drawn.
            float dmax = -INFINITY;
            for (int k = 0; k < HALF; ++k) {
                const int kk = kh + k;
                if (kk >= K) break;
                dmax = fmaxf(dmax, srow[k] + s_lp[kk]);
            }
            x_d[half][sl] = dmax;
        }
        __syncthreads();
        if (cell >= 0) {
            const int kh = kb + half * HALF;
            const float* srow = sc + sl * SS + half * HALF;
            const float dm = fmaxf(x_d[0][sl], x_d[1][sl]);
            // with f the relative factor of bf16_bound and D the distance below
            // dm: the winner is within the noise width of dm, so the condition
            // D > width + f (2|dm| + D + 60) + margins is D > thr
            const float f = (0x1p-17f + (float)(2 * ws.lay_nnz[slot] + 8) * 0x1p-23f) * 1.01f;
            const float adm = fabsf(dm);
            const float thr = ((kGumbelHi - kGumbelLo) + f * (2.0f * adm + 60.0f) +
                               ((float)kNearTie + fmaxf(a.refine_tol, 0.0f)) * (adm + 20.0f) + 1.0f) /
                              (1.0f - f);
            const float cut = dm - thr;
            // four clusters per Philox call; constant indices keep the words
            // in registers
#pragma unroll
            for (int k4 = 0; k4 < HALF; k4 += 4) {
                if (kh + k4 >= K) continue;
                bool any = false;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kk = kh + k4 + q;
                    if (kk < K && srow[k4 + q] + s_lp[kk] >= cut) any = true;
                    if (a.dbg && kk < K && K + 2 <= a.dbg_stride)
                        put_dbg(a.dbg, a.dbg64, (int64_t)cell * a.dbg_stride + kk, (double)srow[k4 + q]);
                }
                if (!any) continue;
                const Words w = philox(ws.seed, (uint32_t)cell, (uint32_t)((kh + k4) >> 2), a.step, kGumbelC, 0u);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kk = kh + k4 + q;
                    if (kk >= K) continue;
                    const float s = srow[k4 + q];
                    const float lp = s_lp[kk];
                    if (s + lp < cut) continue;
                    top.add(lp + s + gumbel32(w.w[q]), s, lp, kk);
                }
            }
        }
    }
    // the two halves of each slot: the upper half hands its best two to the
    // lower, which merges them in cluster order (lower half first, as a single
    // thread scanning the clusters in order would)
    if (half == 1) {
        x_t1[sl] = top.t1; x_t2[sl] = top.t2; x_a1[sl] = top.a1; x_a2[sl] = top.a2;
        x_p1[sl] = top.p1; x_p2[sl] = top.p2; x_k1[sl] = top.k1;
    }
    __syncthreads();
    if (!SUB && (half == 1 || cell < 0)) return;
    if (SUB) {
        // the score tile is free: the block's (row, place) histogram of the
        // fused pass takes its place (visible after the next barrier)
        uint32_t(*ph)[kPlaces] = reinterpret_cast<uint32_t(*)[kPlaces]>(lds);
        const int rows = sa.rsplit ? 4 : 2;
        for (int q = t; q < rows * kPlaces; q += kMfmaThreads) ph[q / kPlaces][q % kPlaces] = 0;
    }
    int sv = -1, cv = 0;
    if (half == 0 && cell >= 0) {
        // column groups alternate halves, so the merged order differs from a scan
        // only among exactly equal values: ties keep the lower cluster index, as
        // here the strict comparisons keep the earlier value and the lower half's
        // clusters of a group precede the upper half's.  With several groups
        // (K > 16 NT) an upper-half cluster can precede a lower-half one of the
        // next group; a tie between them resolves to the lower index explicitly.
        {
            const float u1 = x_t1[sl], u2 = x_t2[sl];
            const int uk = x_k1[sl];
            if (u1 > top.t1 || (u1 == top.t1 && uk < top.k1)) {
                // the upper half's best wins; the runner-up is the better of the
                // lower half's best and the upper half's second
                const float o1 = top.t1, oa = top.a1, op = top.p1;
                top.t2 = o1 > u2 ? o1 : u2;
                top.a2 = o1 > u2 ? oa : x_a2[sl];
                top.p2 = o1 > u2 ? op : x_p2[sl];
                top.t1 = u1; top.a1 = x_a1[sl]; top.p1 = x_p1[sl]; top.k1 = uk;
            } else if (u1 > top.t2) {
                top.t2 = u1; top.a2 = x_a1[sl]; top.p2 = x_p1[sl];
            }
        }
        bool uncertain = false;
        if (K >= 2) {
            const int nnz = ws.lay_nnz[slot];
            const float bnd = bf16_bound(top.a1, top.p1, nnz) + bf16_bound(top.a2, top.p2, nnz);
            const float near = (float)kNearTie * fmaxf(1.0f, fabsf(top.t1));
            if (top.t1 - top.t2 <= bnd + near || (top.t1 - top.t2) / fmaxf(1.0f, fabsf(top.t1)) < a.refine_tol)
                uncertain = true;
        }
        a.c_new[cell] = top.k1;
        // an uncertain decision is re-scored in FP64: by k_refine, or with the
        // fused sub-cluster pass by k_mov_span, which serves that cell's queue
        // entry (flagged) before its sub-cluster draw
        if (!SUB && uncertain) {
            const int q = atomicAdd(&ws.st->n_refine, 1);
            if (q < ws.N) ws.refine[q] = (uint32_t)cell | kRefineCluster;
        }

        if (SUB) {
            // the fused sub-cluster pass: a cell whose certified new label is
            // the block's cluster draws its sub-label here; any other goes to
            // the queue that k_mov_span serves
            const uint32_t i = (uint32_t)cell;
            if (!uncertain && top.k1 == L && L < K) {
                const bool reset = ws.reset[L] != 0;
                double dd = 0.0;
                if (reset) {
                    sv = (int)(philox(ws.seed, i, 0u, sa.step, kResub, 0u).w[0] >> 31);
                } else {
                    // the tail's part of the difference, in entry order, eight
                    // entries' loads in flight at a time
                    const double* dfull = ws.lay_dfull + (int64_t)L * ws.G;
                    double df = s_dfd[sl];
                    const int64_t tb = tbase + s_tbo[sl], te = tbase + s_teo[sl];
                    for (int64_t e0 = tb; e0 < te; e0 += 8) {
                        uint32_t en[8];
                        double dv[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int64_t e = e0 + q < te ? e0 + q : te - 1;
                            en[q] = staged ? t_ent[e - tbase] : ws.lay_tail[e];
                        }
#pragma unroll
                        for (int q = 0; q < 8; ++q) dv[q] = dfull[en[q] & 0xFFFFu];
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            if (e0 + q < te) df = fma((double)(en[q] >> 16), dv[q], df);
                    }
                    const double* lw = ws.lay_sw + 4 * (int64_t)L;
                    const SubWeights w{lw[0], lw[1], lw[2], lw[3]};
                    const int old_code = s_old[sl];
                    const int code = (old_code >> 1) == L ? 1 + (old_code & 1) : 0;
                    sv = sub_draw(ws.seed, i, sa.step, kGumbelS, w, code, sub_noise(ws.seed, i, sa.step, kGumbelS), df, &dd);
                }
                sa.cs_new[i] = (uint8_t)sv;
                atomicAdd(&s_ncnt[sv], 1u);
                if (sa.rsplit) {
                    cv = (int)(philox(ws.seed, i, 0u, sa.rs_step, kRSplit, 0u).w[0] >> 31);
                    ws.rbits[i] = (uint8_t)cv;
                    atomicAdd(&s_ncnt[2 + cv], 1u);
                }
                if (ws.subdd) ws.subdd[i] = reset ? __builtin_nan("") : dd;
            } else {
                const int q = atomicAdd(&ws.st->n_mov, 1);
                if (q < ws.N) ws.mov[q] = i | (uncertain ? kRefineCluster : 0u);
            }
        }
    }
    if constexpr (SUB) {
        if (half == 0) {
            s_sub[sl] = (int8_t)sv;
            s_coin[sl] = (uint8_t)cv;
        }
        __syncthreads();                       // the labels are in; the score tile is free
        const bool rs = sa.rsplit != 0;
        const int rows = rs ? 4 : 2;
        uint32_t(*phist)[kPlaces] = reinterpret_cast<uint32_t(*)[kPlaces]>(lds);   // (cleared above)
        // the statistics of wavefront w's row tiles 2w, 2w + 1, as in the
        // pass of laysub.hip: operand byte e of lane group g stands for cell
        // 32 w + 16 (e >> 2) + 4 g + (e & 3); mask row r of that cell
        const int r = lane & 15, g = lane >> 4;
        long amask;
        {
            uint64_t mk = 0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int c = 32 * wave + 16 * (e >> 2) + 4 * g + (e & 3);
                const int svc = s_sub[c], cvc = s_coin[c];
                const bool on = r < 2 ? svc == r : r < 4 && rs && svc >= 0 && cvc == r - 2;
                if (on) mk |= (uint64_t)1 << (8 * e);
            }
            amask = (long)mk;
        }
        int rc128[4];
        {
            const int svc = lane < 32 ? s_sub[32 * wave + lane] : -1;
            const int cvc = lane < 32 ? s_coin[32 * wave + lane] : 0;
#pragma unroll
            for (int row = 0; row < 4; ++row) {
                const bool on = row < 2 ? svc == row : rs && svc >= 0 && cvc == row - 2;
                rc128[row] = 128 * __popcll(__ballot(on));
            }
        }
        long sel[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = 16 * h + r;
            sel[h] = g == (q >> 3) ? (long)((uint64_t)1 << (8 * (q & 7))) : 0;
        }
        // (the lane's chunk offset formed again from the thread index, which an
        // empty asm hides from the compiler: otherwise the value from the
        // prologue is kept, or spilled, across the whole kernel)
        uint32_t tx = threadIdx.x;
        asm volatile("" : "+v"(tx));
        const uint32_t doff2 = (uint32_t)(((tx >> 6) * 2) * 64 + (tx & 63)) * 16;
        if (rs) chunk_stats<4>(dense, doff2, D, amask, sel, rc128, phist, g, r);
        else chunk_stats<2>(dense, doff2, D, amask, sel, rc128, phist, g, r);
        // the tail entries of the drawn cells, every other one per half: a
        // gene among L's first kPlaces places goes to the histogram, any
        // other straight to the statistics
        {
            const int svc = s_sub[sl], cvc = s_coin[sl];
            if (cell >= 0 && svc >= 0) {
                const uint16_t* rank = ws.lay_rank + (int64_t)L * ws.G;
                unsigned long long* srow = ws.ssub + (int64_t)(2 * L + svc) * ws.G;
                unsigned long long* crow = rs ? ws.rssub + (int64_t)(2 * L + cvc) * ws.G : nullptr;
                // eight entries' ranks in flight at a time
                const int64_t tb = tbase + s_tbo[sl], te = tbase + s_teo[sl];
                for (int64_t e0 = tb + half; e0 < te; e0 += 16) {
                    uint32_t en[8];
                    int p[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int64_t e = e0 + 2 * q < te ? e0 + 2 * q : e0;
                        en[q] = staged ? t_ent[e - tbase] : ws.lay_tail[e];
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q) p[q] = rank[en[q] & 0xFFFFu];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        if (e0 + 2 * q >= te) break;
                        const uint32_t x = en[q] >> 16;
                        if (p[q] < kPlaces) {
                            atomicAdd(&phist[svc][p[q]], x);
                            if (rs) atomicAdd(&phist[2 + cvc][p[q]], x);
                        } else {
                            atomicAdd(&srow[en[q] & 0xFFFFu], (unsigned long long)x);
                            if (rs) atomicAdd(&crow[en[q] & 0xFFFFu], (unsigned long long)x);
                        }
                    }
                }
            }
        }
        __syncthreads();
        uint32_t* part = ws.lay_part + (int64_t)b * ws.lay_pw;
        for (int q = t; q < rows * kPlaces; q += kMfmaThreads) part[q] = phist[q / kPlaces][q % kPlaces];
        if (t < 2 && s_ncnt[t]) atomicAdd(&ws.nsub[2 * L + t], (unsigned long long)s_ncnt[t]);
        if (rs && t < 2 && s_ncnt[2 + t]) atomicAdd(&ws.rnsub[2 * L + t], (unsigned long long)s_ncnt[2 + t]);
    }
}

template <int NT, bool SUB>
static void launch_nt(const Ws& ws, const AssignArgs& a, const SubArgs& sa, hipStream_t s)
{
    hipLaunchKernelGGL((k_assign_bf16<NT, SUB>), dim3((unsigned)ws.nblk_cap), dim3(kMfmaThreads), mfma_lds_bytes(NT), s,
                       ws, a, sa);
}

template <int NT>
static hipError_t configure_nt()
{
    hipError_t e = hipFuncSetAttribute((const void*)k_assign_bf16<NT, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)mfma_lds_bytes(NT));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_assign_bf16<NT, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)mfma_lds_bytes(NT));
    return e;
}

// Allow the dynamic LDS size of every variant on the current device.
hipError_t configure_assign_bf16()
{
    hipError_t e = configure_nt<1>();
    if (e == hipSuccess) e = configure_nt<2>();
    if (e == hipSuccess) e = configure_nt<3>();
    if (e == hipSuccess) e = configure_nt<4>();
    return e;
}

// The column-tile count is fixed at launch while K lives on the device: the
// host passes the last K it has seen (k_hint); if K has grown beyond it the
// kernel loops over column groups.  With the fused sub-cluster pass (sub not
// null) the digit columns count too.
void launch_assign_bf16(const Ws& ws, const AssignArgs& a, const SubArgs* sub, hipStream_t s)
{
    const int k_hint = (a.k_hint > 0 ? a.k_hint : ws.k_max) + (sub ? kSubDigits : 0);
    const int nt = k_hint <= 16 ? 1 : k_hint <= 32 ? 2 : k_hint <= 48 ? 3 : 4;
    const SubArgs none{};
    if (sub) {
        // (with rsplit, the redraw of the same sweep has cleared rssub / rnsub)
        switch (nt) {
        case 1: launch_nt<1, true>(ws, a, *sub, s); break;
        case 2: launch_nt<2, true>(ws, a, *sub, s); break;
        case 3: launch_nt<3, true>(ws, a, *sub, s); break;
        default: launch_nt<4, true>(ws, a, *sub, s); break;
        }
        return;
    }
    switch (nt) {
    case 1: launch_nt<1, false>(ws, a, none, s); break;
    case 2: launch_nt<2, false>(ws, a, none, s); break;
    case 3: launch_nt<3, false>(ws, a, none, s); break;
    default: launch_nt<4, false>(ws, a, none, s); break;
    }
}

}  // namespace dpmm
