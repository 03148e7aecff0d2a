// assign_mfma.hip -- the cluster draw (eq. 4, third line) with the cluster
// log-likelihoods on the matrix cores: S = X L^T for a block of cells, X their
// UMI counts (eq. 26) and L = log theta split as hi + lo in BF16.
//
//   * counts <= 256 are exact in BF16; a larger count x is stored as xa (x
//     with its low bits cleared to keep 8 significant bits, exact in BF16)
//     and the rest (x - xa) log theta is added in FP32;
//   * products of a count and a BF16 value are exact in FP32; the MFMA
//     accumulates in FP32 (v_mfma_f32_16x16x32_bf16, gfx950);
//   * S = X hi^T + X lo^T, |log theta - hi - lo| <= 2^-17 |log theta|.
//
// A workgroup of 4 wavefronts owns one block of kBlkCells cells of the
// blocked layout; wavefront w owns cells 64w .. 64w + 63 (4 row tiles of 16).
// For each chunk of 64 genes: the workgroup stages the hi/lo chunk of
// log theta cluster-major, reads the chunk's segment with coalesced 16-byte
// loads and writes each pre-encoded entry (BF16 value at its LDS byte offset)
// into the dense tile, then each wavefront issues 2 k-steps x 4 row tiles x
// Nt column tiles x 2 (hi, lo) MFMAs, and the entries are cleared again.  The
// next chunk's entries and log theta rows are loaded into registers while
// this chunk computes.  Counts above 256 come from a static per-block list
// whose FP32 corrections are added to the scores.
// The cell's lane then takes the Gumbel-max over the K scores with a
// certified rounding bound; close decisions are queued for the FP64 re-score.
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4_t;

constexpr int kMfmaThreads = kBlkCells;       // 256: one thread per cell
constexpr int kMfmaRow = kBlkRow;             // BF16 elements per LDS tile row (padded)
constexpr int kPrefetch = 2;                  // segment entries held in registers: 2 x 4 per thread
constexpr int kMaxChunks = (65535 + kBlkGenes - 1) / kBlkGenes;

__host__ __device__ constexpr size_t mfma_main_bytes(int nt)
{
    // A tile (256 cells) + hi/lo B tiles, or the FP32 score tile reusing them
    return (size_t)(kBlkCells * kMfmaRow * 2 + 2 * 16 * nt * kMfmaRow * 2) >
                   (size_t)kBlkCells * (16 * nt + 1) * 4
               ? (size_t)(kBlkCells * kMfmaRow * 2 + 2 * 16 * nt * kMfmaRow * 2)
               : (size_t)kBlkCells * (16 * nt + 1) * 4;
}
__host__ __device__ constexpr size_t mfma_lds_bytes(int nt) { return mfma_main_bytes(nt); }

// one pre-encoded entry into the tile: BF16 value at its byte offset
__device__ inline void put(char* tile, uint32_t en) { *reinterpret_cast<uint16_t*>(tile + (en >> 16)) = (uint16_t)en; }
__device__ inline void wipe(char* tile, uint32_t en) { *reinterpret_cast<uint16_t*>(tile + (en >> 16)) = 0; }

__device__ inline float gumbel32(uint32_t w) { return -logf(-logf(unit23f(w))); }

// rounding bound of a split-BF16 score: representation 2^-17, FP32
// accumulation over nsteps MFMA k-steps (with slack for the 32-term products
// inside each), FP32 overflow corrections and the FP32 Gumbel noise
__device__ inline float bf16_bound(float acc, float lp, int nsteps)
{
    return ((float)(nsteps + 40) * 0x1p-24f + 0x1p-17f) * (fabsf(acc) + fabsf(lp) + 20.0f) + 1e-5f;
}

// hi/lo rows of log theta for one chunk: 2 x 16 NT rows x 64 genes, one
// 16-byte piece per thread and r
template <int NT>
struct BRows {
    uint4 v[NT];
};

__device__ inline void brow_slot(int idx, int nt, int& tbl, int& row, int& sg)
{
    const int per = 16 * nt * (kBlkGenes / 8);
    tbl = idx / per;
    const int rem = idx - tbl * per;
    row = rem / (kBlkGenes / 8);
    sg = rem % (kBlkGenes / 8);
}

template <int NT>
__device__ inline BRows<NT> load_brows(const Ws& ws, int kb, int jj, int t)
{
    BRows<NT> b;
#pragma unroll
    for (int r = 0; r < NT; ++r) {
        int tbl, row, sg;
        brow_slot(t + r * kMfmaThreads, NT, tbl, row, sg);
        b.v[r] = *reinterpret_cast<const uint4*>((tbl ? ws.llo : ws.lhi) + (int64_t)(kb + row) * ws.Gpad +
                                                 jj * kBlkGenes + sg * 8);
    }
    return b;
}

template <int NT>
__device__ inline void store_brows(const BRows<NT>& b, uint16_t* bhi, uint16_t* blo, int t)
{
#pragma unroll
    for (int r = 0; r < NT; ++r) {
        int tbl, row, sg;
        brow_slot(t + r * kMfmaThreads, NT, tbl, row, sg);
        *reinterpret_cast<uint4*>((tbl ? blo : bhi) + row * kMfmaRow + sg * 8) = b.v[r];
    }
}

// raw buffer resource over n bytes at p (gfx9 descriptor word 3); loads past
// n bytes return zeros
constexpr int kBufWord3 = 0x00020000;
constexpr int kOutOfRange = 0x7FFFFFF0;
__device__ inline __amdgpu_buffer_rsrc_t buffer_of(const void* p, uint32_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)n, kBufWord3);
}

// The first kPrefetch x 4 entries of a segment [f0, f1), through a buffer
// resource over the block's entries: a lane past the segment end asks for an
// offset beyond the resource and reads the entry 0, which writes into a
// padding column.  The loads are unconditional, so the compiler waits for
// exactly the loads a use needs.
__device__ inline void load_segment(__amdgpu_buffer_rsrc_t ent, uint32_t f0, uint32_t f1, int t, uint4 (&seg)[kPrefetch])
{
#pragma unroll
    for (int r = 0; r < kPrefetch; ++r) {
        const uint32_t q = f0 + 4 * t + 4 * kMfmaThreads * r;
        const int off = q < f1 ? (int)(4 * q) : kOutOfRange;
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(ent, off, 0, 0);
        seg[r] = make_uint4(v[0], v[1], v[2], v[3]);
    }
}

template <int NT>
__global__ void __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(NT <= 2 ? 3 : 2))) k_assign_bf16(Ws ws, AssignArgs a)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    uint16_t* atile = reinterpret_cast<uint16_t*>(lds);
    uint16_t* bhi = atile + kBlkCells * kMfmaRow;
    uint16_t* blo = bhi + 16 * NT * kMfmaRow;
    float* sc = reinterpret_cast<float*>(lds);                         // epilogue alias
    constexpr int SS = 16 * NT + 1;

    const int K = ws.st->K;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int blk = blockIdx.x;
    const int64_t i = (int64_t)blk * kBlkCells + t;
    const bool valid = i < ws.N;
    const int64_t* soff = ws.blk_off + (int64_t)blk * ws.nch;
    const uint32_t* bent = ws.blk_ent + soff[0];       // this block's entries, 32-bit offsets below
    const __amdgpu_buffer_rsrc_t bres = buffer_of(bent, (uint32_t)(4 * (soff[ws.nch] - soff[0])));
    // the block's segment offsets, relative to its first entry, once into LDS
    __shared__ uint32_t s_off[kMaxChunks + 1];
    for (int q = t; q <= ws.nch; q += kMfmaThreads) s_off[q] = (uint32_t)(soff[q] - soff[0]);
    __syncthreads();

    float t1 = -INFINITY, t2 = -INFINITY, a1 = 0.f, a2 = 0.f, p1 = 0.f, p2 = 0.f;
    int k1 = 0;
    const int nsteps = 2 * ws.nch;

    for (int kb = 0; kb < K; kb += 16 * NT) {
        floatx4_t acc[4][NT];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[m][n] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        __syncthreads();
        // clear the tile once; afterwards only written entries are cleared
        for (int g = 0; g < kMfmaRow; g += 8)
            *reinterpret_cast<uint4*>(atile + t * kMfmaRow + g) = make_uint4(0, 0, 0, 0);

        // Software pipeline with two register stages (chunks of even and odd
        // index): a stage holds its chunk's B rows and first kPrefetch x 4
        // segment entries; after the chunk has been multiplied and its
        // entries wiped, the stage is reloaded with the chunk two ahead, so
        // the loads have a whole chunk to arrive.  The chunk count is even
        // and past the last chunk the index is clamped, so no stage is
        // conditional and every path issues the same loads.
        const int last = ws.nch - 1;
        BRows<NT> nb0 = load_brows<NT>(ws, kb, 0, t);
        uint4 sg0[kPrefetch];
        uint32_t f00 = s_off[0], f01 = s_off[1];
        load_segment(bres, f00, f01, t, sg0);
        BRows<NT> nb1 = load_brows<NT>(ws, kb, 1, t);
        uint4 sg1[kPrefetch];
        uint32_t f10 = s_off[1], f11 = s_off[2];
        load_segment(bres, f10, f11, t, sg1);
        char* tileb = reinterpret_cast<char*>(atile);

        auto phase = [&](int j, BRows<NT>& nb, uint4 (&sg)[kPrefetch], uint32_t& f0, uint32_t& f1)
            __attribute__((always_inline)) {
            __syncthreads();
            // commit chunk j: B rows to LDS, entries into the tile
            store_brows<NT>(nb, bhi, blo, t);
#pragma unroll
            for (int r = 0; r < kPrefetch; ++r) {
                put(tileb, sg[r].x); put(tileb, sg[r].y); put(tileb, sg[r].z); put(tileb, sg[r].w);
            }
            for (uint32_t q = f0 + 4 * t + 4 * kMfmaThreads * kPrefetch; q < f1; q += 4 * kMfmaThreads) {
                const uint4 v = *reinterpret_cast<const uint4*>(bent + q);
                put(tileb, v.x); put(tileb, v.y); put(tileb, v.z); put(tileb, v.w);
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int col = 32 * s + 8 * (lane >> 4);
                bf16x8_t af[4];
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    af[m] = *reinterpret_cast<const bf16x8_t*>(atile + (64 * wave + 16 * m + (lane & 15)) * kMfmaRow + kBlkLead + col);
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const bf16x8_t bh = *reinterpret_cast<const bf16x8_t*>(bhi + (16 * n + (lane & 15)) * kMfmaRow + col);
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[m], bh, acc[m][n], 0, 0, 0);
                }
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const bf16x8_t bl = *reinterpret_cast<const bf16x8_t*>(blo + (16 * n + (lane & 15)) * kMfmaRow + col);
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[m], bl, acc[m][n], 0, 0, 0);
                }
            }
            __syncthreads();
            // clear the written entries (the first ones are still in the stage)
#pragma unroll
            for (int r = 0; r < kPrefetch; ++r) {
                wipe(tileb, sg[r].x); wipe(tileb, sg[r].y); wipe(tileb, sg[r].z); wipe(tileb, sg[r].w);
            }
            for (uint32_t q = f0 + 4 * t + 4 * kMfmaThreads * kPrefetch; q < f1; q += 4 * kMfmaThreads) {
                const uint4 v = *reinterpret_cast<const uint4*>(bent + q);
                wipe(tileb, v.x); wipe(tileb, v.y); wipe(tileb, v.z); wipe(tileb, v.w);
            }
            // reload the stage with the chunk two ahead
            const int jn = min(j + 2, last);
            f0 = s_off[jn];
            f1 = s_off[jn + 1];
            nb = load_brows<NT>(ws, kb, jn, t);
            load_segment(bres, f0, f1, t, sg);
        };
        for (int j = 0; j < ws.nch; j += 2) {
            phase(j, nb0, sg0, f00, f01);
            phase(j + 1, nb1, sg1, f10, f11);
        }
        __syncthreads();
        // scores through LDS: lane l holds, for row tile m and column tile n,
        // cells 64w + 16m + 4(l/16) + j (j < 4) against cluster 16n + l%16
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    sc[(64 * wave + 16 * m + 4 * (lane >> 4) + q) * SS + 16 * n + (lane & 15)] = acc[m][n][q];
        __syncthreads();
        // FP32 corrections of the counts above 256 (static list of this block)
        for (int64_t o = ws.ovf_off[blk] + t; o < ws.ovf_off[blk + 1]; o += kMfmaThreads) {
            const uint2 ov = ws.ovf_ent[o];
            const int cell = (int)(ov.x & 0xFFu);
            const int g = (int)(ov.x >> 8);
            const float xb = (float)ov.y;
            const float* lrow = ws.lc32 + (int64_t)g * ws.kpad + kb;
            for (int k = 0; k < 16 * NT && kb + k < K; ++k) atomicAdd(&sc[cell * SS + k], xb * lrow[k]);
        }
        __syncthreads();
        if (valid) {
            // four clusters per Philox call; constant word indices keep the
            // words in registers
            for (int k4 = 0; k4 < 16 * NT && kb + k4 < K; k4 += 4) {
                const Words w = philox(ws.seed, (uint32_t)i, (uint32_t)((kb + k4) >> 2), a.step, kGumbelC, 0u);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kk = kb + k4 + q;
                    if (kk >= K) break;
                    const float s = sc[t * SS + k4 + q];
                    const float lp = (float)ws.logpi[kk];
                    const float v = lp + s + gumbel32(w.w[q]);
                    if (a.dbg && K + 2 <= a.dbg_stride) put_dbg(a.dbg, a.dbg64, i * a.dbg_stride + kk, (double)s);
                    if (v > t1) {
                        t2 = t1; a2 = a1; p2 = p1;
                        t1 = v; a1 = s; p1 = lp; k1 = kk;
                    } else if (v > t2) {
                        t2 = v; a2 = s; p2 = lp;
                    }
                }
            }
        }
    }
    if (!valid) return;
    bool uncertain = false;
    if (K >= 2) {
        const float bnd = bf16_bound(a1, p1, nsteps) + bf16_bound(a2, p2, nsteps);
        const float near = (float)kNearTie * fmaxf(1.0f, fabsf(t1));
        if (t1 - t2 <= bnd + near || (t1 - t2) / fmaxf(1.0f, fabsf(t1)) < a.refine_tol) uncertain = true;
    }
    a.c_new[i] = k1;
    if (uncertain) {
        const int q = atomicAdd(&ws.st->n_refine, 1);
        if (q < ws.N) ws.refine[q] = (uint32_t)i | kRefineCluster;
    }
}

template <int NT>
static void launch_nt(const Ws& ws, const AssignArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_assign_bf16<NT>, dim3((unsigned)ws.nblk), dim3(kMfmaThreads), mfma_lds_bytes(NT), s, ws, a);
}

// Allow the dynamic LDS size of every variant on the current device.
hipError_t configure_assign_bf16()
{
    hipError_t e = hipFuncSetAttribute((const void*)k_assign_bf16<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)mfma_lds_bytes(1));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_assign_bf16<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)mfma_lds_bytes(2));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_assign_bf16<3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)mfma_lds_bytes(3));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_assign_bf16<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)mfma_lds_bytes(4));
    return e;
}

// The column-tile count is fixed at launch while K lives on the device: the
// host passes the last K it has seen (k_hint); if K has grown beyond it the
// kernel loops over column groups.
void launch_assign_bf16(const Ws& ws, const AssignArgs& a, hipStream_t s)
{
    const int k_hint = a.k_hint > 0 ? a.k_hint : ws.k_max;
    const int nt = k_hint <= 16 ? 1 : k_hint <= 32 ? 2 : k_hint <= 48 ? 3 : 4;
    switch (nt) {
    case 1: launch_nt<1>(ws, a, s); break;
    case 2: launch_nt<2>(ws, a, s); break;
    case 3: launch_nt<3>(ws, a, s); break;
    default: launch_nt<4>(ws, a, s); break;
    }
}

}  // namespace dpmm
