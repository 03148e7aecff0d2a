// prep.hip -- preprocessing of a count matrix before the sampler.  The paper
// keeps the genes of largest standard deviation across cells (Section 3);
// these kernels give the exact per-gene moments for that ranking and restrict
// a cell-major CSR to a chosen set of genes, renumbered.
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

constexpr int kPrepThreads = 256;
constexpr int kScanThreads = 1024;

// sum_i x_iu and sum_i x_iu^2 as exact 64-bit integers (entries with a gene
// outside [0, G) or a count < 1 are skipped)
__global__ void __launch_bounds__(kPrepThreads) k_gene_moments(const int32_t* __restrict__ col,
                                                               const int32_t* __restrict__ val, int64_t nnz, int32_t G,
                                                               unsigned long long* sum, unsigned long long* sumsq)
{
    for (int64_t e = (int64_t)blockIdx.x * kPrepThreads + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kPrepThreads) {
        const int32_t u = col[e];
        const int32_t x = val[e];
        if (u < 0 || u >= G || x < 1) continue;
        atomicAdd(&sum[u], (unsigned long long)x);
        atomicAdd(&sumsq[u], (unsigned long long)x * (unsigned long long)x);
    }
}

__device__ inline bool kept(const int32_t* map, int32_t G, int32_t u) { return u >= 0 && u < G && map[u] >= 0; }

// one wavefront per row: the number of kept entries, into out_ptr[row + 1]
__global__ void __launch_bounds__(kPrepThreads) k_filter_count(const int64_t* __restrict__ row_ptr,
                                                               const int32_t* __restrict__ col, int64_t N, int32_t G,
                                                               const int32_t* __restrict__ map, int64_t* out_ptr)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (kPrepThreads / 64) + (threadIdx.x >> 6);
    if (row >= N) return;
    int n = 0;
    for (int64_t e = row_ptr[row] + lane; e < row_ptr[row + 1]; e += 64) n += kept(map, G, col[e]) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
    if (lane == 0) {
        out_ptr[row + 1] = n;
        if (row == 0) out_ptr[0] = 0;
    }
}

// inclusive scan of v[1..n] in place, one workgroup: each thread sums a
// contiguous chunk, the chunk totals are scanned in LDS, then each thread
// rewrites its chunk
__global__ void __launch_bounds__(kScanThreads) k_scan_one_block(int64_t* v, int64_t n)
{
    __shared__ int64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t chunk = (n + kScanThreads - 1) / kScanThreads;
    const int64_t b = 1 + t * chunk, e = min(n + 1, b + chunk);
    int64_t s = 0;
    for (int64_t q = b; q < e; ++q) s += v[q];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int64_t add = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int64_t q = b; q < e; ++q) {
        run += v[q];
        v[q] = run;
    }
}

// one wavefront per row: the kept entries in their order, genes renumbered
__global__ void __launch_bounds__(kPrepThreads) k_filter_fill(const int64_t* __restrict__ row_ptr,
                                                              const int32_t* __restrict__ col,
                                                              const int32_t* __restrict__ val, int64_t N, int32_t G,
                                                              const int32_t* __restrict__ map,
                                                              const int64_t* __restrict__ out_ptr, int32_t* col_out,
                                                              int32_t* val_out)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (kPrepThreads / 64) + (threadIdx.x >> 6);
    if (row >= N) return;
    int64_t dst = out_ptr[row];
    const uint64_t below = (1ull << lane) - 1ull;
    for (int64_t base = row_ptr[row]; base < row_ptr[row + 1]; base += 64) {
        const int64_t e = base + lane;
        const bool k = e < row_ptr[row + 1] && kept(map, G, col[e]);
        const uint64_t mask = __ballot(k);
        if (k) {
            const int64_t at = dst + __popcll(mask & below);
            col_out[at] = map[col[e]];
            val_out[at] = val[e];
        }
        dst += __popcll(mask);
    }
}

// ---------------------------------------------------------------------------
// The k genes of largest standard deviation.  The population variance of gene
// u is B_u / N^2 with B_u = N sum x^2 - (sum x)^2, an integer below 2^127 for
// N < 2^31 and 64-bit moments; N^2 is common to all genes, so ranking by B in
// exact 128-bit arithmetic ranks the standard deviations exactly.  Equal B go
// to the lower gene.
// ---------------------------------------------------------------------------
typedef unsigned __int128 u128;

__device__ inline u128 variance_numerator(unsigned long long s, unsigned long long q, uint64_t n)
{
    return (u128)n * (u128)q - (u128)s * (u128)s;
}

// rank of gene g = the genes before it in (B descending, gene ascending); the
// genes of rank < k are flagged in map (1, else -1).  Each workgroup walks all
// genes in tiles of kPrepThreads, the tile's B in LDS.
__global__ void __launch_bounds__(kPrepThreads) k_gene_rank(const unsigned long long* __restrict__ sum,
                                                            const unsigned long long* __restrict__ sumsq, int32_t G,
                                                            uint64_t n, int32_t k, int32_t* map, double* std_out)
{
    __shared__ unsigned long long thi[kPrepThreads], tlo[kPrepThreads];
    const int g = blockIdx.x * kPrepThreads + threadIdx.x;
    const u128 bg = g < G ? variance_numerator(sum[g], sumsq[g], n) : 0;
    int above = 0;
    for (int h0 = 0; h0 < G; h0 += kPrepThreads) {
        const int h = h0 + threadIdx.x;
        const u128 bh = h < G ? variance_numerator(sum[h], sumsq[h], n) : 0;
        __syncthreads();
        thi[threadIdx.x] = (unsigned long long)(bh >> 64);
        tlo[threadIdx.x] = (unsigned long long)bh;
        __syncthreads();
        const int m = min(kPrepThreads, G - h0);
        for (int j = 0; j < m; ++j) {
            const u128 b = ((u128)thi[j] << 64) | (u128)tlo[j];
            above += (b > bg || (b == bg && h0 + j < g)) ? 1 : 0;
        }
    }
    if (g >= G) return;
    map[g] = above < k ? 1 : -1;
    if (std_out) {
        const double v = (double)(unsigned long long)(bg >> 64) * 0x1p64 + (double)(unsigned long long)bg;
        std_out[g] = sqrt(v) / (double)n;
    }
}

// one workgroup: the flagged genes numbered 0, 1, ... in gene order
__global__ void __launch_bounds__(kScanThreads) k_gene_places(int32_t* map, int32_t G)
{
    __shared__ int32_t part[kScanThreads];
    const int t = threadIdx.x;
    const int chunk = (G + kScanThreads - 1) / kScanThreads;
    const int b = t * chunk, e = min(G, b + chunk);
    int c = 0;
    for (int u = b; u < e; ++u) c += map[u] > 0 ? 1 : 0;
    part[t] = c;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int add = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int at = part[t] - c;
    for (int u = b; u < e; ++u) map[u] = map[u] > 0 ? at++ : -1;
}

void launch_top_genes(const unsigned long long* sum, const unsigned long long* sumsq, int32_t G, int64_t N, int32_t k,
                      int32_t* map, double* std_out, hipStream_t s)
{
    const unsigned blocks = (unsigned)((G + kPrepThreads - 1) / kPrepThreads);
    hipLaunchKernelGGL(k_gene_rank, dim3(blocks), dim3(kPrepThreads), 0, s, sum, sumsq, G, (uint64_t)N, k, map,
                       std_out);
    hipLaunchKernelGGL(k_gene_places, dim3(1), dim3(kScanThreads), 0, s, map, G);
}

void launch_gene_moments(const int32_t* col, const int32_t* val, int64_t nnz, int32_t G, unsigned long long* sum,
                         unsigned long long* sumsq, hipStream_t s)
{
    launch_zero(sum, sizeof(unsigned long long) * (size_t)G, s);
    launch_zero(sumsq, sizeof(unsigned long long) * (size_t)G, s);
    if (nnz <= 0) return;
    int64_t blocks = (nnz + kPrepThreads - 1) / kPrepThreads;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_gene_moments, dim3((unsigned)blocks), dim3(kPrepThreads), 0, s, col, val, nnz, G, sum, sumsq);
}

void launch_filter_count(const int64_t* row_ptr, const int32_t* col, int64_t N, int32_t G, const int32_t* map,
                         int64_t* out_ptr, hipStream_t s)
{
    const unsigned blocks = (unsigned)((N + kPrepThreads / 64 - 1) / (kPrepThreads / 64));
    hipLaunchKernelGGL(k_filter_count, dim3(blocks), dim3(kPrepThreads), 0, s, row_ptr, col, N, G, map, out_ptr);
    hipLaunchKernelGGL(k_scan_one_block, dim3(1), dim3(kScanThreads), 0, s, out_ptr, N);
}

void launch_filter_fill(const int64_t* row_ptr, const int32_t* col, const int32_t* val, int64_t N, int32_t G,
                        const int32_t* map, const int64_t* out_ptr, int32_t* col_out, int32_t* val_out, hipStream_t s)
{
    const unsigned blocks = (unsigned)((N + kPrepThreads / 64 - 1) / (kPrepThreads / 64));
    hipLaunchKernelGGL(k_filter_fill, dim3(blocks), dim3(kPrepThreads), 0, s, row_ptr, col, val, N, G, map, out_ptr,
                       col_out, val_out);
}

}  // namespace dpmm
