// layout.hip -- the blocked copy of the count matrix read by the matrix-core
// kernel, built once at init from the packed rows.
//
// Cells are taken in blocks of kBlkCells (in input order) and genes in chunks
// of kBlkGenes.  Segment (b, j) holds every entry of block b's cells whose
// gene is in chunk j, ordered by cell then gene, as
//   cell-in-block (8 bits) | gene-in-chunk << 8 (6 bits) | count << 16,
// and is padded with zero entries (count 0) to a multiple of four, so that a
// workgroup reads a chunk's entries with coalesced 16-byte loads and scatters
// them into its dense tile entry by entry, with no per-cell walk.
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

constexpr int kLayThreads = kBlkCells;   // one thread per cell of the block

// entries of each (block, chunk), padded to a multiple of 4
__global__ void __launch_bounds__(kLayThreads) k_seg_count(Ws ws)
{
    extern __shared__ uint32_t cnt[];    // [nch]
    const int b = blockIdx.x;
    for (int j = threadIdx.x; j < ws.nch; j += kLayThreads) cnt[j] = 0;
    __syncthreads();
    const int64_t i = (int64_t)b * kBlkCells + threadIdx.x;
    if (i < ws.N) {
        for (int64_t p = ws.roff[i]; p < ws.roff[i + 1]; ++p) {
            const uint32_t en = ws.ent[p];
            if (en >> 16) atomicAdd(&cnt[(en & 0xFFFFu) / kBlkGenes], 1u);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < ws.nch; j += kLayThreads)
        ws.blk_off[(int64_t)b * ws.nch + j] = (int64_t)((cnt[j] + 3u) & ~3u);
}

// write the entries: per chunk, a workgroup-wide exclusive scan of the cells'
// entry counts gives each cell its place in the segment
__global__ void __launch_bounds__(kLayThreads) k_seg_fill(Ws ws)
{
    __shared__ uint32_t scan[kLayThreads];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t i = (int64_t)b * kBlkCells + t;
    int64_t pos = i < ws.N ? ws.roff[i] : 0;
    const int64_t end = i < ws.N ? ws.roff[i + 1] : 0;
    uint32_t* out = const_cast<uint32_t*>(ws.blk_ent);
    for (int j = 0; j < ws.nch; ++j) {
        const int hi = (j + 1) * kBlkGenes;
        uint32_t n = 0;
        for (int64_t p = pos; p < end; ++p) {
            const uint32_t en = ws.ent[p];
            if ((int)(en & 0xFFFFu) >= hi) break;
            if (en >> 16) ++n;
        }
        scan[t] = n;
        __syncthreads();
        for (int off = 1; off < kLayThreads; off <<= 1) {
            const uint32_t add = t >= off ? scan[t - off] : 0u;
            __syncthreads();
            scan[t] += add;
            __syncthreads();
        }
        const uint32_t total = scan[kLayThreads - 1];
        const int64_t seg = ws.blk_off[(int64_t)b * ws.nch + j];
        const int64_t seg_end = ws.blk_off[(int64_t)b * ws.nch + j + 1];
        int64_t w = seg + scan[t] - n;
        while (pos < end) {
            const uint32_t en = ws.ent[pos];
            const int g = (int)(en & 0xFFFFu);
            if (g >= hi) break;
            if (en >> 16) {
                out[w++] = (uint32_t)t | ((uint32_t)(g - j * kBlkGenes) << 8) | (en & 0xFFFF0000u);
            }
            ++pos;
        }
        for (int64_t q = seg + total + t; q < seg_end; q += kLayThreads) out[q] = 0u;
        __syncthreads();
    }
}

void launch_build_blocked(const Ws& ws, int64_t* tile_sums, hipStream_t s)
{
    const int64_t nseg = (int64_t)ws.nblk * ws.nch;
    hipLaunchKernelGGL(k_seg_count, dim3(ws.nblk), dim3(kLayThreads), sizeof(uint32_t) * (size_t)ws.nch, s, ws);
    launch_exclusive_scan(ws.blk_off, nseg, tile_sums, s);
    hipLaunchKernelGGL(k_seg_fill, dim3(ws.nblk), dim3(kLayThreads), 0, s, ws);
}

}  // namespace dpmm
