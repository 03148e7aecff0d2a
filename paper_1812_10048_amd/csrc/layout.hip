// layout.hip -- the blocked copy of the count matrix read by the matrix-core
// kernel, built once at init from the packed rows.
//
// Cells are taken in blocks of kBlkCells (in input order) and genes in chunks
// of kBlkGenes.  Segment (b, j) holds every entry of block b's cells whose
// gene is in chunk j, ordered by cell then gene.  Since the counts never
// change, each entry is stored ready for the kernel's scatter into its dense
// BF16 tile in LDS:
//   low 16 bits   BF16 value of the count (of its top 8 significant bits
//                 when the count exceeds 256),
//   high 16 bits  byte offset of (cell, gene) in the tile.
// Each tile row starts with kBlkLead padding columns, so the entry 0 (BF16
// zero at byte offset 0) writes into a padding column: segments are padded to
// a multiple of four with it, so the scatter needs no test, and a load that
// returns zeros is harmless too.  Counts above
// 256 also go to a per-block list (cell, gene, count - head) whose FP32
// corrections the kernel adds to the scores.
//
// The order of the entries inside a segment is free (each carries its own
// offset).  The matrix-core kernel reads a segment with 16-byte loads, thread
// t taking positions 1024r + 4t + c, so one wavefront store instruction
// (wave w, r, c) writes the entries at 1024r + 256w + 4l + c, l < 64.  A
// last pass reorders each segment so that such an instruction writes
// entries of distinct LDS banks: the entries are taken round-robin over the
// banks (rank within the bank, then bank) and dealt to the store
// instructions in turn, 64 consecutive ones each.
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

constexpr int kLayThreads = kBlkCells;   // one thread per cell of the block

__device__ inline uint32_t count_head(uint32_t x)
{
    if (x <= 256u) return x;
    const int sh = (32 - __clz((int)x)) - 8;
    return (x >> sh) << sh;
}

__device__ inline uint32_t encode_entry(int cell, int g_local, uint32_t x)
{
    // a count with at most 8 significant bits is exact in FP32 and BF16
    const uint32_t bf = __float_as_uint((float)count_head(x)) >> 16;
    const uint32_t off = (uint32_t)(cell * kBlkRow + kBlkLead + g_local) * 2u;
    return bf | (off << 16);
}

// entries of each (block, chunk), padded to a multiple of 4, and the number
// of counts above 256 of each block
__global__ void __launch_bounds__(kLayThreads) k_seg_count(Ws ws)
{
    extern __shared__ uint32_t cnt[];    // [nch]
    __shared__ uint32_t novf;
    const int b = blockIdx.x;
    for (int j = threadIdx.x; j < ws.nch; j += kLayThreads) cnt[j] = 0;
    if (threadIdx.x == 0) novf = 0;
    __syncthreads();
    const int64_t i = (int64_t)b * kBlkCells + threadIdx.x;
    if (i < ws.N) {
        for (int64_t p = ws.roff[i]; p < ws.roff[i + 1]; ++p) {
            const uint32_t en = ws.ent[p];
            const uint32_t x = en >> 16;
            // (a gene past G is invalid input, reported by the row check)
            if (!x || (en & 0xFFFFu) >= (uint32_t)ws.G) continue;
            atomicAdd(&cnt[(en & 0xFFFFu) / kBlkGenes], 1u);
            if (count_head(x) != x) atomicAdd(&novf, 1u);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < ws.nch; j += kLayThreads)
        ws.blk_off[(int64_t)b * ws.nch + j] = (int64_t)((cnt[j] + 3u) & ~3u);
    if (threadIdx.x == 0) ws.ovf_off[b] = (int64_t)novf;
}

__device__ inline uint32_t block_exclusive(uint32_t v, uint32_t* scan, uint32_t* total)
{
    const int t = threadIdx.x;
    scan[t] = v;
    __syncthreads();
    for (int off = 1; off < kLayThreads; off <<= 1) {
        const uint32_t add = t >= off ? scan[t - off] : 0u;
        __syncthreads();
        scan[t] += add;
        __syncthreads();
    }
    const uint32_t incl = scan[t];
    *total = scan[kLayThreads - 1];
    __syncthreads();
    return incl - v;
}

// write the entries: per chunk, a workgroup-wide exclusive scan of the cells'
// entry counts gives each cell its place in the segment
__global__ void __launch_bounds__(kLayThreads) k_seg_fill(Ws ws)
{
    __shared__ uint32_t scan[kLayThreads];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t i = (int64_t)b * kBlkCells + t;
    const int64_t rb = i < ws.N ? ws.roff[i] : 0;
    const int64_t end = i < ws.N ? ws.roff[i + 1] : 0;
    uint32_t* out = const_cast<uint32_t*>(ws.blk_ent);
    const uint32_t pad = 0u;                 // zero into cell 0's first padding column
    int64_t pos = rb;
    for (int j = 0; j < ws.nch; ++j) {
        const int hi = (j + 1) * kBlkGenes;
        uint32_t n = 0;
        for (int64_t p = pos; p < end; ++p) {
            const uint32_t en = ws.ent[p];
            if ((int)(en & 0xFFFFu) >= hi) break;
            if (en >> 16) ++n;
        }
        uint32_t total;
        const uint32_t before = block_exclusive(n, scan, &total);
        const int64_t seg = ws.blk_off[(int64_t)b * ws.nch + j];
        const int64_t seg_end = ws.blk_off[(int64_t)b * ws.nch + j + 1];
        int64_t w = seg + before;
        while (pos < end) {
            const uint32_t en = ws.ent[pos];
            const int g = (int)(en & 0xFFFFu);
            if (g >= hi) break;
            if (en >> 16) out[w++] = encode_entry(t, g - j * kBlkGenes, en >> 16);
            ++pos;
        }
        for (int64_t q = seg + total + t; q < seg_end; q += kLayThreads) out[q] = pad;
    }
    // counts above 256: (cell | gene << 8, count - head)
    uint32_t n = 0;
    for (int64_t p = rb; p < end; ++p) {
        const uint32_t x = ws.ent[p] >> 16;
        if (x && count_head(x) != x) ++n;
    }
    uint32_t total;
    int64_t w = ws.ovf_off[b] + block_exclusive(n, scan, &total);
    for (int64_t p = rb; p < end; ++p) {
        const uint32_t en = ws.ent[p];
        const uint32_t x = en >> 16;
        if (x && count_head(x) != x)
            ws.ovf_ent[w++] = make_uint2((uint32_t)t | ((en & 0xFFFFu) << 8), x - count_head(x));
    }
}

constexpr int kBalThreads = 256;
constexpr int kLdsBanks = 64;                       // LDS banks of 4 bytes
constexpr int kMaxSegEntries = kBlkCells * kBlkGenes;   // every (cell, gene) of a block and chunk

// position of the k-th entry of the round-robin order in a segment of n
// entries (n a multiple of 4): the store instructions (r, w, c) in turn, each
// with m = min(64, (n - 1024r - 256w) / 4) lanes
__device__ inline uint32_t balanced_position(uint32_t k, uint32_t n)
{
    uint32_t base = 0;
    for (uint32_t rw = 0;; ++rw) {
        const uint32_t start = 256u * rw;     // 1024r + 256w
        const uint32_t m = min(64u, (n - start) / 4u);
        if (k < base + 4u * m) {
            const uint32_t c = (k - base) / m;
            const uint32_t l = (k - base) - c * m;
            return start + 4u * l + c;
        }
        base += 4u * m;
    }
}

__global__ void __launch_bounds__(kBalThreads) k_seg_balance(Ws ws)
{
    extern __shared__ uint32_t buf[];           // [kMaxSegEntries] the segment
    __shared__ uint32_t cnt[kLdsBanks], rank[kLdsBanks], npad;
    const int64_t sg = blockIdx.x;
    const int64_t b0 = ws.blk_off[sg];
    const uint32_t n = (uint32_t)(ws.blk_off[sg + 1] - b0);
    // (a longer segment only comes from invalid input, reported by the row check)
    if (n == 0 || n > (uint32_t)kMaxSegEntries) return;
    uint32_t* seg = const_cast<uint32_t*>(ws.blk_ent) + b0;
    const int t = threadIdx.x;
    if (t < kLdsBanks) { cnt[t] = 0; rank[t] = 0; }
    if (t == 0) npad = 0;
    for (uint32_t q = t; q < n; q += kBalThreads) buf[q] = seg[q];
    __syncthreads();
    for (uint32_t q = t; q < n; q += kBalThreads) {
        const uint32_t en = buf[q];
        if (en & 0xFFFFu) atomicAdd(&cnt[(en >> 18) & (kLdsBanks - 1)], 1u);
    }
    __syncthreads();
    uint32_t nreal = 0;
    for (int b = 0; b < kLdsBanks; ++b) nreal += cnt[b];
    for (uint32_t q = t; q < n; q += kBalThreads) {
        const uint32_t en = buf[q];
        uint32_t k;
        if (en & 0xFFFFu) {
            const uint32_t b = (en >> 18) & (kLdsBanks - 1);
            const uint32_t r = atomicAdd(&rank[b], 1u);
            // entries before (r, b): min(cnt, r) of every bank, and one of each
            // earlier bank that reaches rank r
            k = 0;
            for (uint32_t b2 = 0; b2 < (uint32_t)kLdsBanks; ++b2)
                k += min(cnt[b2], r) + (b2 < b && cnt[b2] > r ? 1u : 0u);
        } else {
            k = nreal + atomicAdd(&npad, 1u);    // padding (zero) entries last
        }
        seg[balanced_position(k, n)] = en;
    }
}

hipError_t configure_layout()
{
    return hipFuncSetAttribute((const void*)k_seg_balance, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(sizeof(uint32_t) * (size_t)kMaxSegEntries));
}

void launch_build_blocked(const Ws& ws, int64_t* tile_sums, hipStream_t s)
{
    const int64_t nseg = (int64_t)ws.nblk * ws.nch;
    hipLaunchKernelGGL(k_seg_count, dim3(ws.nblk), dim3(kLayThreads), sizeof(uint32_t) * (size_t)ws.nch, s, ws);
    launch_exclusive_scan(ws.blk_off, nseg, tile_sums, s);
    launch_exclusive_scan(ws.ovf_off, ws.nblk, tile_sums, s);
    hipLaunchKernelGGL(k_seg_fill, dim3(ws.nblk), dim3(kLayThreads), 0, s, ws);
    hipLaunchKernelGGL(k_seg_balance, dim3((unsigned)nseg), dim3(kBalThreads), sizeof(uint32_t) * (size_t)kMaxSegEntries,
                       s, ws);
}

}  // namespace dpmm
