// bookkeeping.hip -- packing of the count matrix, initial labels, the integer
// sufficient statistics (step a4), compaction of empty clusters and label
// relabelling.
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

// ---------------------------------------------------------------------------
// Packing.  Each CSR row becomes a run of 32-bit entries (gene | count << 16)
// padded to a multiple of four entries so that rows start 16-byte aligned.
// ---------------------------------------------------------------------------

__global__ void k_padded_lengths(const int64_t* __restrict__ row_ptr, int64_t N, int64_t* __restrict__ out,
                                 DevState* st)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t len = row_ptr[i + 1] - row_ptr[i];
    if (len < 0 || (i == 0 && row_ptr[0] != 0)) atomicAdd(&st->data_error, 1);
    out[i] = len < 0 ? 0 : ((len + 3) & ~(int64_t)3);
}

// Exclusive scan of v[0..n) in place, v[n] = total.  Three phases over
// tiles of kScanTile elements.
constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 16;
constexpr int kScanTile = kScanThreads * kScanPerThread;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* lds, int64_t* total)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int64_t add = t >= off ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    const int64_t incl = lds[t];
    *total = lds[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_tiles(int64_t* __restrict__ v, int64_t n, int64_t* __restrict__ tile_sums, const int32_t* gate)
{
    __shared__ int64_t lds[kScanThreads];
    if (gate && !*gate) return;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
    int64_t loc[kScanPerThread];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanPerThread; ++j) {
        const int64_t idx = base + j;
        loc[j] = idx < n ? v[idx] : 0;
        s += loc[j];
    }
    int64_t total;
    int64_t run = block_exclusive_scan(s, lds, &total);
#pragma unroll
    for (int j = 0; j < kScanPerThread; ++j) {
        const int64_t idx = base + j;
        if (idx < n) v[idx] = run;
        run += loc[j];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_tile_sums(int64_t* __restrict__ tile_sums, int64_t ntiles, const int32_t* gate)
{
    __shared__ int64_t lds[kScanThreads];
    if (gate && !*gate) return;
    int64_t carry = 0;
    for (int64_t b = 0; b < ntiles; b += kScanThreads) {
        const int64_t idx = b + threadIdx.x;
        const int64_t v = idx < ntiles ? tile_sums[idx] : 0;
        int64_t total;
        const int64_t ex = block_exclusive_scan(v, lds, &total);
        if (idx < ntiles) tile_sums[idx] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) tile_sums[ntiles] = carry;
}

__global__ void k_scan_add(int64_t* __restrict__ v, int64_t n, const int64_t* __restrict__ tile_sums,
                           int64_t ntiles, const int32_t* gate)
{
    if (gate && !*gate) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] += tile_sums[i / kScanTile];
    if (i == 0) v[n] = tile_sums[ntiles];
}

void launch_exclusive_scan(int64_t* v, int64_t n, int64_t* tile_sums, hipStream_t s, const int32_t* gate)
{
    const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles > 0)
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, v, n, tile_sums, gate);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(kScanThreads), 0, s, tile_sums, ntiles, gate);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 256) / 256)), dim3(256), 0, s, v, n, tile_sums, ntiles, gate);
}

// One wavefront per row: validate (columns strictly increasing and < G,
// counts in [1, 65535]) and write the packed, padded row.
__global__ void k_pack_rows(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ val, int64_t N, int32_t G, int64_t nnz,
                            const int64_t* __restrict__ roff, uint32_t* __restrict__ ent, DevState* st)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= N) return;
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    const int64_t o = roff[row], pe = roff[row + 1];
    int bad = 0;
    if (b < 0 || e > nnz || e < b) bad = 1;
    for (int64_t j = lane; j < pe - o; j += 64) {
        uint32_t packed = kPadEntry;
        if (!bad && j < e - b) {
            const int32_t g = col[b + j];
            const int32_t x = val[b + j];
            if (g < 0 || g >= G || x < 1 || x > 65535) bad = 1;
            if (j > 0 && col[b + j - 1] >= g) bad = 1;
            packed = (uint32_t)(g & 0xFFFF) | ((uint32_t)(x & 0xFFFF) << 16);
        }
        ent[o + j] = packed;
    }
    if (bad) atomicAdd(&st->data_error, 1);
}

void launch_pack(const int64_t* row_ptr, const int32_t* col, const int32_t* val, int64_t N, int32_t G, int64_t nnz,
                 int64_t* roff, int64_t* tile_sums, uint32_t* ent, DevState* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_padded_lengths, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, row_ptr, N, roff, st);
    launch_exclusive_scan(roff, N, tile_sums, s);
    hipLaunchKernelGGL(k_pack_rows, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, row_ptr, col, val, N, G, nnz,
                       roff, ent, st);
}

// ---------------------------------------------------------------------------
// Initial labels: one cluster, or k_init clusters drawn uniformly.
// ---------------------------------------------------------------------------
__global__ void k_init_labels(Ws ws, int32_t k_init, int32_t* __restrict__ c, uint8_t* __restrict__ cs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ws.N) {
        int32_t k = 0;
        if (k_init > 1) {
            const Words w = philox(ws.seed, (uint32_t)i, 0u, 0u, kInit, 0u);
            k = (int32_t)(((uint64_t)w.w[0] * (uint64_t)k_init) >> 32);
        }
        c[i] = k;
        cs[i] = 0;
    }
    if (i < ws.k_max) ws.reset[i] = i < (k_init < 1 ? 1 : k_init) ? 1 : 0;
    if (i == 0) ws.st->K = k_init < 1 ? 1 : k_init;
}

void launch_init_labels(const Ws& ws, int32_t k_init, int32_t* c, uint8_t* cs, hipStream_t s)
{
    const int64_t n = ws.N > ws.k_max ? ws.N : ws.k_max;
    hipLaunchKernelGGL(k_init_labels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ws, k_init, c, cs);
}

// ---------------------------------------------------------------------------
// Step a4: integer statistics n_{k,r} and s_{k,r,u}.
//
// The cells are first counting-sorted by group q = 2k + r (labels c, cbar):
// per-workgroup LDS histograms, one global reservation per (workgroup,
// group), then a scatter of cell indices into `perm`.  The group sizes are
// n_{k,r} themselves.  The statistics kernel then walks `perm` in ranges of
// kStatCells cells: a range holds one or a few runs of equal group, each
// accumulated in an LDS histogram over genes and flushed with one 64-bit
// atomic per non-zero gene.  Integer sums are exact, so the order of the
// additions (and the order of cells within a group) does not matter.
// `perm` also serves as the processing order of the next sweep, which keeps
// the cells of one cluster together.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 1024;
constexpr int kSortPerThread = 8;
constexpr int kSortCellsPerBlock = kSortThreads * kSortPerThread;
constexpr int kStatThreads = 256;
constexpr int kStatCells = 2048;
constexpr int kStatMaxGenes = 16384;

__device__ inline int sort_group(int32_t k, uint8_t r, int by_cluster) { return by_cluster ? k : 2 * k + (r & 1); }

// A thread's cells are i = b0 + j kSortThreads + t, j < kSortPerThread; their
// labels are loaded together, one round trip per pass.
struct SortCells {
    int32_t g[kSortPerThread];      // group of each cell, -1 if none
    uint32_t old[kSortPerThread];   // with c_prev: 1 + the old sub-label if the cell stays in its cluster, else 0
};

__device__ inline SortCells load_groups(const Ws& ws, const int32_t* __restrict__ c, const uint8_t* __restrict__ cs,
                                        int by_cluster, int64_t b0, int64_t b1,
                                        const int32_t* __restrict__ c_prev = nullptr)
{
    SortCells sc;
    int32_t k[kSortPerThread], kp[kSortPerThread];
    uint8_t r[kSortPerThread];
    const bool want_old = c_prev && by_cluster;
#pragma unroll
    for (int j = 0; j < kSortPerThread; ++j) {
        const int64_t i = b0 + (int64_t)j * kSortThreads + threadIdx.x;
        k[j] = i < b1 ? c[i] : -1;
        r[j] = (i < b1 && (!by_cluster || want_old)) ? cs[i] : 0;
        kp[j] = (i < b1 && want_old) ? c_prev[i] : -1;
    }
#pragma unroll
    for (int j = 0; j < kSortPerThread; ++j) {
        sc.g[j] = (k[j] >= 0 && k[j] < ws.k_max) ? sort_group(k[j], r[j], by_cluster) : -1;
        sc.old[j] = (sc.g[j] >= 0 && want_old && kp[j] == k[j]) ? 1u + (r[j] & 1u) : 0u;
    }
    return sc;
}

__global__ void __launch_bounds__(kSortThreads) k_group_count(Ws ws, const int32_t* __restrict__ c,
                                                              const uint8_t* __restrict__ cs, int by_cluster,
                                                              const int32_t* gate)
{
    extern __shared__ uint32_t hist[];   // [groups]
    if (gate && !*gate) return;
    const int ng = by_cluster ? ws.k_max : 2 * ws.k_max;
    for (int q = threadIdx.x; q < ng; q += kSortThreads) hist[q] = 0;
    const int64_t b0 = (int64_t)blockIdx.x * kSortCellsPerBlock;
    const int64_t b1 = min(ws.N, b0 + kSortCellsPerBlock);
    const SortCells sc = load_groups(ws, c, cs, by_cluster, b0, b1);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortPerThread; ++j)
        if (sc.g[j] >= 0) atomicAdd(&hist[sc.g[j]], 1u);
    __syncthreads();
    for (int q = threadIdx.x; q < ng; q += kSortThreads)
        if (hist[q]) atomicAdd(&ws.grp_cnt[q], (int32_t)hist[q]);
}

// exclusive scan of the group sizes; with groups (k, r) the sizes are n_{k,r}
__global__ void __launch_bounds__(kSortThreads) k_group_scan(Ws ws, int by_cluster, const int32_t* gate)
{
    __shared__ int32_t lds[kSortThreads];
    if (gate && !*gate) return;
    const int ng = by_cluster ? ws.k_max : 2 * ws.k_max;
    int32_t carry = 0;
    for (int base = 0; base < ng; base += kSortThreads) {
        const int q = base + threadIdx.x;
        const int32_t v = q < ng ? ws.grp_cnt[q] : 0;
        lds[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kSortThreads; off <<= 1) {
            const int32_t add = (int)threadIdx.x >= off ? lds[threadIdx.x - off] : 0;
            __syncthreads();
            lds[threadIdx.x] += add;
            __syncthreads();
        }
        if (q < ng) {
            ws.grp_off[q] = carry + lds[threadIdx.x] - v;
            ws.grp_cur[q] = 0;
            if (!by_cluster) ws.nsub[q] = (unsigned long long)v;
        }
        carry += lds[kSortThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) ws.grp_off[ng] = carry;
}

__global__ void __launch_bounds__(kSortThreads) k_group_scatter(Ws ws, const int32_t* __restrict__ c,
                                                                const uint8_t* __restrict__ cs, int by_cluster,
                                                                const int32_t* __restrict__ c_prev,
                                                                const int32_t* gate)
{
    extern __shared__ uint32_t lds_u[];      // [groups] counts, then [groups] bases
    if (gate && !*gate) return;
    const int ng = by_cluster ? ws.k_max : 2 * ws.k_max;
    uint32_t* cnt = lds_u;
    uint32_t* base = lds_u + ng;
    for (int q = threadIdx.x; q < ng; q += kSortThreads) cnt[q] = 0;
    const int64_t b0 = (int64_t)blockIdx.x * kSortCellsPerBlock;
    const int64_t b1 = min(ws.N, b0 + kSortCellsPerBlock);
    const SortCells sc = load_groups(ws, c, cs, by_cluster, b0, b1, c_prev);
    // the row offsets depend only on the cell: loaded with the labels
    int64_t r0[kSortPerThread], r1[kSortPerThread];
#pragma unroll
    for (int j = 0; j < kSortPerThread; ++j) {
        const int64_t i = b0 + (int64_t)j * kSortThreads + threadIdx.x;
        r0[j] = sc.g[j] >= 0 ? ws.roff[i] : 0;
        r1[j] = sc.g[j] >= 0 ? ws.roff[i + 1] : 0;
    }
    __syncthreads();
    // pass 1: block-local counts; pass 2: one reservation per group; pass 3: ranks
#pragma unroll
    for (int j = 0; j < kSortPerThread; ++j)
        if (sc.g[j] >= 0) atomicAdd(&cnt[sc.g[j]], 1u);
    __syncthreads();
    for (int q = threadIdx.x; q < ng; q += kSortThreads) {
        base[q] = cnt[q] ? (uint32_t)(ws.grp_off[q] + atomicAdd(&ws.grp_cur[q], (int32_t)cnt[q])) : 0u;
        cnt[q] = 0;
    }
    __syncthreads();
    uint32_t pos[kSortPerThread];
#pragma unroll
    for (int j = 0; j < kSortPerThread; ++j)
        pos[j] = sc.g[j] >= 0 ? base[sc.g[j]] + atomicAdd(&cnt[sc.g[j]], 1u) : 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < kSortPerThread; ++j) {
        const int64_t i = b0 + (int64_t)j * kSortThreads + threadIdx.x;
        if (pos[j] < (uint32_t)ws.N) {
            ws.perm[pos[j]] = (int32_t)i;
            // the row of the sorted cell, so that kernels walking the sorted
            // order reach it (and the cell's old membership) with one load;
            // a padded row holds at most 65536 entries, below bit 30
            ws.srow[pos[j]] = make_uint4((uint32_t)i, (uint32_t)r0[j], (uint32_t)(r0[j] >> 32),
                                         (uint32_t)(r1[j] - r0[j]) | (sc.old[j] << kSrowOldShift));
        }
    }
}

// group of a sorted position (binary search over the group offsets)
__device__ inline int group_of(const Ws& ws, int64_t pos, int ng)
{
    int lo = 0, hi = ng;   // grp_off[lo] <= pos < grp_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ws.grp_off[mid] <= pos) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(kStatThreads) k_stats_sorted(Ws ws)
{
    extern __shared__ uint32_t hist[];       // [G]
    const int G = ws.G;
    const int ng = 2 * ws.st->K;
    const int64_t p0 = (int64_t)blockIdx.x * kStatCells;
    const int64_t p1 = min(ws.N, p0 + kStatCells);
    if (p0 >= p1) return;
    for (int u = threadIdx.x; u < G; u += kStatThreads) hist[u] = 0;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int q = group_of(ws, p0, ng); q < ng && ws.grp_off[q] < p1; ++q) {
        const int64_t r0 = max(p0, (int64_t)ws.grp_off[q]);
        const int64_t r1 = min(p1, (int64_t)ws.grp_off[q + 1]);
        if (r0 >= r1) continue;
        __syncthreads();
        for (int64_t p = r0 + wave; p < r1; p += kStatThreads / 64) {
            const int32_t i = ws.perm[p];
            const int64_t b = ws.roff[i], e = ws.roff[i + 1];
            for (int64_t j = b + lane; j < e; j += 64) {
                const uint32_t en = ws.ent[j];
                const uint32_t x = en >> 16;
                if (x) atomicAdd(&hist[en & 0xFFFFu], x);
            }
        }
        __syncthreads();
        unsigned long long* row = ws.ssub + (int64_t)q * G;
        for (int u = threadIdx.x; u < G; u += kStatThreads) {
            const uint32_t v = hist[u];
            if (v) {
                atomicAdd(&row[u], (unsigned long long)v);
                hist[u] = 0;
            }
        }
    }
}

// Fallback for very wide gene panels: one wavefront per cell, 64-bit atomics.
__global__ void k_stats_atomic(Ws ws, const int32_t* __restrict__ c, const uint8_t* __restrict__ cs)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int K = ws.st->K;
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < ws.N; i += waves) {
        const int32_t k = c[i];
        if (k < 0 || k >= K) continue;
        const int64_t grp = 2 * (int64_t)k + (cs[i] & 1);
        unsigned long long* row = ws.ssub + grp * ws.G;
        const int64_t b = ws.roff[i], e = ws.roff[i + 1];
        for (int64_t j = b + lane; j < e; j += 64) {
            const uint32_t en = ws.ent[j];
            const uint32_t x = en >> 16;
            if (x) atomicAdd(&row[en & 0xFFFF], (unsigned long long)x);
        }
    }
}

// Zero n 32-bit words with a kernel (unlike a memset node it is safe in a
// captured graph, and its launch error is seen by hipGetLastError).
__global__ void k_zero_words(uint32_t* p, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0u;
}

void launch_zero(void* p, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<uint32_t*>(p), n);
}

void launch_sort(const Ws& ws, const int32_t* c, const uint8_t* cs, int by_cluster, hipStream_t s,
                 bool counts_cleared, const int32_t* c_prev, const int32_t* gate)
{
    const int ng = by_cluster ? ws.k_max : 2 * ws.k_max;
    if (!counts_cleared) launch_zero(ws.grp_cnt, sizeof(int32_t) * (size_t)ng, s);
    const unsigned sb = (unsigned)((ws.N + kSortCellsPerBlock - 1) / kSortCellsPerBlock);
    hipLaunchKernelGGL(k_group_count, dim3(sb), dim3(kSortThreads), sizeof(uint32_t) * (size_t)ng, s, ws, c, cs,
                       by_cluster, gate);
    hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(kSortThreads), 0, s, ws, by_cluster, gate);
    hipLaunchKernelGGL(k_group_scatter, dim3(sb), dim3(kSortThreads), 2 * sizeof(uint32_t) * (size_t)ng, s, ws, c,
                       cs, by_cluster, c_prev, gate);
}

void launch_stats(const Ws& ws, const int32_t* c, const uint8_t* cs, hipStream_t s)
{
    launch_zero(ws.ssub, sizeof(unsigned long long) * 2 * (size_t)ws.k_max * (size_t)ws.G, s);
    launch_sort(ws, c, cs, 0, s);
    if (ws.G <= kStatMaxGenes) {
        const unsigned blocks = (unsigned)((ws.N + kStatCells - 1) / kStatCells);
        hipLaunchKernelGGL(k_stats_sorted, dim3(blocks), dim3(kStatThreads), sizeof(uint32_t) * (size_t)ws.G, s, ws);
    } else {
        int64_t blocks = (ws.N + 3) / 4;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_stats_atomic, dim3((unsigned)blocks), dim3(256), 0, s, ws, c, cs);
    }
}

// ---------------------------------------------------------------------------
// Compaction: drop clusters with no cells, keep the order of the others, and
// move statistics and reset flags with them (one workgroup).  After a sweep
// the consumed reset flags are cleared and a cluster of >= 2 cells with an
// empty sub-cluster is flagged; after a split/merge the flags move along.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kMaxClusters) k_compact(Ws ws, int after_sweep)
{
    extern __shared__ int32_t lds_map[];      // [k_max]
    __shared__ int32_t s_wave[kMaxClusters / 64];
    const int t = threadIdx.x;
    // thread t holds cluster t's counts (k_max <= kMaxClusters = blockDim.x),
    // loaded before K is known
    unsigned long long n0 = 0, n1 = 0;
    if (t < ws.k_max) {
        n0 = ws.nsub[2 * t];
        n1 = ws.nsub[2 * t + 1];
    }
    const int K = ws.st->K;
    // the map in order: a cluster with cells takes the number of clusters
    // with cells below it (a workgroup-wide exclusive count)
    const bool live = t < K && (n0 + n1) > 0;
    int nk;
    const int pos = block_exclusive_count(live, s_wave, &nk);
    if (t < K) lds_map[t] = live ? pos : -1;
    // changed: a cluster with cells takes a new index, so labels must be
    // rewritten; dropping empty clusters at the end renumbers nobody (the
    // barrier also publishes the map)
    const int changed = __syncthreads_or(live && pos != t);
    const int G = ws.G;
    // the coin-half statistics of a coming random split move with the rest
    const bool rs = ws.rssub && ws.st->rs_live;
    if (changed || nk < K) {
        // (lds_map is uniform over the workgroup: only a row that moves costs
        // a barrier, which orders it before a later move into its place)
        for (int k = 0; k < K; ++k) {
            const int j = lds_map[k];
            if (j < 0 || j == k) continue;
            for (int u = t; u < 2 * G; u += blockDim.x)
                ws.ssub[(int64_t)2 * j * G + u] = ws.ssub[(int64_t)2 * k * G + u];
            if (rs)
                for (int u = t; u < 2 * G; u += blockDim.x)
                    ws.rssub[(int64_t)2 * j * G + u] = ws.rssub[(int64_t)2 * k * G + u];
            if (t < 2) ws.nsub[2 * j + t] = ws.nsub[2 * k + t];
            if (rs && t < 2) ws.rnsub[2 * j + t] = ws.rnsub[2 * k + t];
            if (t == 0) ws.reset[j] = ws.reset[k];
            __syncthreads();
        }
        for (int k = nk; k < K; ++k) {
            for (int u = t; u < 2 * G; u += blockDim.x) ws.ssub[(int64_t)2 * k * G + u] = 0;
            if (rs)
                for (int u = t; u < 2 * G; u += blockDim.x) ws.rssub[(int64_t)2 * k * G + u] = 0;
            if (t < 2) ws.nsub[2 * k + t] = 0;
            if (rs && t < 2) ws.rnsub[2 * k + t] = 0;
            if (t == 0) ws.reset[k] = 0;
        }
        __syncthreads();
    }
    for (int k = t; k < K; k += blockDim.x) {
        ws.relab_c[2 * k] = lds_map[k];
        ws.relab_c[2 * k + 1] = lds_map[k];
        ws.relab_s[2 * k] = 0xFF;
        ws.relab_s[2 * k + 1] = 0xFF;
    }
    if (after_sweep) {
        // cluster t (if it has cells) is now cluster lds_map[t] < nk, with the
        // counts this thread holds; the flags from nk on are 0 (two disjoint
        // sets of indices)
        if (t < ws.k_max && t >= nk) ws.reset[t] = 0;
        if (t < K && lds_map[t] >= 0) ws.reset[lds_map[t]] = (n0 + n1 >= 2 && (n0 == 0 || n1 == 0)) ? 1 : 0;
    }
    if (t == 0) {
        ws.st->K = nk;
        ws.st->has_new = 0;
        ws.st->relabel = changed;
        if (changed) ws.st->relabels += 1;
        if (ws.k_hint) __hip_atomic_store(ws.k_hint, nk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// The Gibbs step over K + 1 clusters (eq. 4): append cluster K empty, with
// its sub-labels to be drawn at random; the redraw then gives it a prior theta
// and the alpha component of pi.  Nothing is appended at k_max.
__global__ void k_extend(Ws ws)
{
    const int K = ws.st->K;
    if (K >= ws.k_max) {
        if (threadIdx.x == 0) ws.st->has_new = 0;
        return;
    }
    for (int u = threadIdx.x; u < 2 * ws.G; u += blockDim.x) ws.ssub[(int64_t)2 * K * ws.G + u] = 0;
    if (threadIdx.x == 0) {
        ws.nsub[2 * K] = ws.nsub[2 * K + 1] = 0;
        ws.reset[K] = 1;
        ws.st->K = K + 1;
        ws.st->has_new = 1;
    }
}

void launch_extend(const Ws& ws, hipStream_t s)
{
    hipLaunchKernelGGL(k_extend, dim3(1), dim3(256), 0, s, ws);
}

void launch_compact(const Ws& ws, int after_sweep, hipStream_t s)
{
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(kMaxClusters), sizeof(int32_t) * (size_t)ws.k_max, s, ws, after_sweep);
}

// Apply relab_c / relab_s to every label when the relabel flag is set.
__global__ void k_relabel(Ws ws, int32_t* __restrict__ c, uint8_t* __restrict__ cs)
{
    if (!ws.st->relabel) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ws.N; i += stride) {
        const int32_t k = c[i];
        if (k < 0 || k >= ws.k_max) continue;
        const int q = 2 * k + (cs[i] & 1);
        c[i] = ws.relab_c[q];
        const uint8_t r = ws.relab_s[q];
        if (r != 0xFF) cs[i] = r;
    }
}

void launch_relabel(const Ws& ws, int32_t* c, uint8_t* cs, hipStream_t s)
{
    int64_t blocks = (ws.N + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_relabel, dim3((unsigned)blocks), dim3(256), 0, s, ws, c, cs);
}

// Labels written by the caller: count out-of-range values.
__global__ void k_check_labels(Ws ws, const int32_t* __restrict__ c, const uint8_t* __restrict__ cs, int32_t K)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ws.N) return;
    if (c[i] < 0 || c[i] >= K || cs[i] > 1) atomicAdd(&ws.st->data_error, 1);
}

void launch_check_labels(const Ws& ws, const int32_t* c, const uint8_t* cs, int32_t K, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_labels, dim3((unsigned)((ws.N + 255) / 256)), dim3(256), 0, s, ws, c, cs, K);
}

}  // namespace dpmm
