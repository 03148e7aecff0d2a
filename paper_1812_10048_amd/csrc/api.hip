// api.hip -- host side of the libdpmm C ABI (include/dpmm.h): argument
// checks, workspace carving, and the order in which the kernels of a sweep,
// a split/merge move and the empirical-Bayes step are enqueued.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/dpmm.h"
#include "dpmm_common.hpp"
#include "kernels.hpp"

using namespace dpmm;

namespace {

thread_local char g_err[512] = "";

dpmm_status fail(dpmm_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(DPMM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxTimed = 16384;       // timed stage intervals kept between two reads
constexpr int kTablePadRows = 64;      // spare cluster rows read by its last column group
constexpr int kRelayoutEvery = 8;      // sweeps between checks of the cluster-sorted copy

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
    size_t ent, roff, tiles, c0, c1, cs0, cs1, st, reset, nsub, ssub, beta, lgbeta, logpi, lt64, lc32, ls32, lhi, llo,
        lgrise, subdd, qsub, rbits, rssub, rnsub, refine, perm, srow, grp_cnt, grp_off, grp_cur, nsub_prev, lay_kc,
        lay_pbeg, lay_pcnt, lay_cell, lay_doff, lay_toff, lay_dense, lay_tail, lay_nnz, lay_hcnt, lay_bh, lay_rank, lay_gene, lay_bhi,
        lay_blo, lay_lim, lay_dE, lay_dS, lay_dfull, lay_sw, lay_part, lay_bbeg, lay_sbeg, mov, relab_c, relab_s, sm_logr, sm_acc, mkey, mlist, dm_k, eb_tmp, rd_part, sm_part, total;
};

int32_t num_blocks(int64_t N) { return (int32_t)((N + kBlkCells - 1) / kBlkCells); }
// blocks of the cluster-sorted copy: each cluster's last block may be partial
int32_t lay_blocks(int64_t N, int32_t k_max) { return num_blocks(N) + k_max; }
int32_t lay_cols(int32_t k_max) { return (k_max + kSubDigits + 15) / 16 * 16 + kTablePadRows; }
// words of a block's statistics histogram in the sub-cluster pass over the
// copy: (sub-cluster 0, 1 [, coin 0, 1]) x the places of the dense chunks
int32_t lay_hist_words(uint32_t flags)
{
    return ((flags & kFlagRandomSplit) ? 4 : 2) * kLayDmax * kBlkGenes;
}
// gene chunks of the split-BF16 kernel: an even number, so that its pipeline
// (two register stages, unrolled by two) has no conditional chunk; the chunks
// past G hold no entries and zero log theta
int32_t num_chunks(int32_t G)
{
    const int32_t n = (G + kBlkGenes - 1) / kBlkGenes;
    return (n + 1) / 2 * 2;
}

Layout plan(int64_t N, int32_t G, int64_t nnz, int32_t k_max, int32_t precision, uint32_t flags)
{
    Layout L{};
    const int64_t nnz_pad = nnz + 3 * N;
    const int64_t kpad = (k_max + 15) / 16 * 16;
    const int64_t Gpad = (int64_t)num_chunks(G) * kBlkGenes;
    const int64_t ncand = (int64_t)k_max + (int64_t)k_max * (k_max - 1) / 2;
    const bool blocked = precision == DPMM_SPLIT_BF16;
    const int64_t nbc = blocked ? lay_blocks(N, k_max) : 0;
    const int64_t nslots = nbc * kBlkCells;
    const int64_t ntiles = ((N > nslots ? N : nslots) + 4095) / 4096 + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += align_up(bytes); return at; };
    L.ent = take(4 * (size_t)(nnz_pad + 4));   // + one 16-byte slot of slack
    L.roff = take(8 * (size_t)(N + 1));
    L.tiles = take(8 * (size_t)(ntiles + 1));
    L.c0 = take(4 * (size_t)N);
    L.c1 = take(4 * (size_t)N);
    L.cs0 = take((size_t)N);
    L.cs1 = take((size_t)N);
    L.st = take(sizeof(DevState));
    L.reset = take((size_t)k_max);
    L.nsub = take(16 * (size_t)k_max);
    L.ssub = take(16 * (size_t)k_max * (size_t)G);
    L.beta = take(8 * (size_t)G);
    L.lgbeta = take(8 * (size_t)G);
    L.lgrise = take(8 * (size_t)kRiseTab * (size_t)G);
    L.subdd = take((flags & kFlagSplitQ) ? 8 * (size_t)N : 0);
    L.qsub = take(8 * (size_t)k_max);
    const bool rsplit = (flags & kFlagRandomSplit) != 0;
    L.rbits = take(rsplit ? (size_t)N : 0);
    L.rssub = take(rsplit ? 16 * (size_t)k_max * (size_t)G : 0);
    L.rnsub = take(rsplit ? 16 * (size_t)k_max : 0);
    L.logpi = take(8 * (size_t)k_max);
    L.lt64 = take(24 * (size_t)k_max * (size_t)G);
    L.lc32 = take(4 * ((size_t)G * (size_t)kpad + kTablePadRows));
    L.ls32 = take(8 * (size_t)G * (size_t)k_max);
    L.lhi = take(2 * (size_t)Gpad * (size_t)(kpad + kTablePadRows));
    L.llo = take(2 * (size_t)Gpad * (size_t)(kpad + kTablePadRows));
    L.refine = take(4 * (size_t)N);
    L.perm = take(4 * (size_t)N);
    L.srow = take(16 * (size_t)N);
    L.grp_cnt = take(8 * (size_t)k_max);
    L.grp_off = take(8 * (size_t)k_max + 4);
    L.grp_cur = take(8 * (size_t)k_max);
    L.nsub_prev = take(16 * (size_t)k_max);
    L.lay_kc = take(blocked ? 4 * (size_t)nbc : 0);
    L.lay_pbeg = take(blocked ? 4 * (size_t)nbc : 0);
    L.lay_pcnt = take(blocked ? 4 * (size_t)nbc : 0);
    L.lay_cell = take(blocked ? 4 * (size_t)nslots : 0);
    L.lay_doff = take(blocked ? 8 * (size_t)(nbc + 1) : 0);
    L.lay_toff = take(blocked ? 8 * (size_t)(nslots + 1) : 0);
    // a block's dense chunks cost less than the tail entries they take
    // (kTailCost each), so they hold at most kTailCost bytes per entry, and a
    // block has at most kLayDmax of them; plus one high-plane chunk per block
    const int64_t dense_chunks = std::min<int64_t>((nnz * kTailCost + kDenseChunkBytes - 1) / kDenseChunkBytes + 1,
                                                   nbc * (int64_t)kLayDmax);
    L.lay_dense = take(blocked ? (size_t)kDenseChunkBytes * (size_t)(dense_chunks + nbc) : 0);
    L.lay_tail = take(blocked ? 4 * (size_t)(nnz > 0 ? nnz : 1) : 0);   // at most every entry
    L.lay_nnz = take(blocked ? 2 * (size_t)nslots : 0);
    L.lay_hcnt = take(blocked ? (size_t)nslots : 0);
    L.lay_bh = take(blocked ? (size_t)nbc : 0);
    L.lay_rank = take(blocked ? 2 * (size_t)k_max * (size_t)G : 0);
    L.lay_gene = take(blocked ? 2 * (size_t)k_max * kLayDmax * kBlkGenes : 0);
    L.lay_bhi = take(blocked ? 2 * (size_t)k_max * (size_t)lay_cols(k_max) * kLayDmax * kBlkGenes : 0);
    L.lay_blo = take(blocked ? 2 * (size_t)k_max * (size_t)lay_cols(k_max) * kLayDmax * kBlkGenes : 0);
    L.lay_lim = take(blocked ? 8 * (size_t)k_max * kLayDmax * 2 * 8 * 4 : 0);
    L.lay_dE = take(blocked ? 4 * (size_t)k_max : 0);
    L.lay_dS = take(blocked ? 4 * (size_t)k_max * (kLayDmax + 1) * 8 : 0);
    L.lay_dfull = take(blocked ? 8 * (size_t)k_max * (size_t)G : 0);
    L.lay_sw = take(blocked ? 8 * (size_t)k_max * 4 : 0);
    L.lay_part = take(blocked ? 4 * (size_t)nbc * (size_t)lay_hist_words(flags) : 0);
    L.lay_bbeg = take(blocked ? 4 * (size_t)(k_max + 1) : 0);
    L.lay_sbeg = take(blocked ? 4 * (size_t)(k_max + 1) : 0);
    L.mov = take(blocked ? 4 * (size_t)N : 0);
    L.relab_c = take(8 * (size_t)k_max);
    L.relab_s = take(2 * (size_t)k_max);
    L.sm_logr = take(8 * (size_t)ncand);
    L.sm_acc = take((size_t)ncand);
    L.mkey = take(8 * (size_t)ncand);
    L.mlist = take(4 * (size_t)ncand);
    L.dm_k = take(8 * (size_t)k_max);
    L.eb_tmp = take(8 * ((size_t)k_max + (size_t)G));
    L.rd_part = take(16 * (size_t)(3 * k_max + 1) * (size_t)redraw_tiles(G));
    L.sm_part = take(sizeof(SmPart) * (size_t)k_max * (size_t)sm_tiles(G));
    L.total = o;
    return L;
}

dpmm_status check_args(const dpmm_csr* csr, const dpmm_params* p)
{
    if (!csr || !p) return fail(DPMM_ERR_ARG, "null csr or params");
    if (csr->n_cells < 1 || csr->n_cells >= (1ll << 30)) return fail(DPMM_ERR_ARG, "n_cells must be in [1, 2^30)");
    if (csr->n_genes < 1 || csr->n_genes > 65535) return fail(DPMM_ERR_ARG, "n_genes must be in [1, 65535]");
    if (csr->nnz < 0) return fail(DPMM_ERR_ARG, "nnz must be >= 0");
    if (csr->reserved != 0) return fail(DPMM_ERR_ARG, "reserved field must be 0");
    if (!(p->alpha > 0.0)) return fail(DPMM_ERR_ARG, "alpha must be > 0");
    if (!p->beta_per_gene && !(p->beta > 0.0)) return fail(DPMM_ERR_ARG, "beta must be > 0");
    if (p->k_max < 1 || p->k_max > kMaxClusters) return fail(DPMM_ERR_ARG, "k_max must be in [1, 1024]");
    if (p->k_init < 1 || p->k_init > p->k_max) return fail(DPMM_ERR_ARG, "k_init must be in [1, k_max]");
    if (p->precision < DPMM_FP64 || p->precision > DPMM_SPLIT_BF16) return fail(DPMM_ERR_ARG, "unknown precision");
    if (p->flags & ~(DPMM_FLAG_SPLIT_Q | DPMM_FLAG_NEW_CLUSTER | DPMM_FLAG_RANDOM_SPLIT))
        return fail(DPMM_ERR_ARG, "unknown flags");
    return DPMM_OK;
}

}  // namespace

struct dpmm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t N = 0, nnz = 0;
    int32_t G = 0, k_max = 0, precision = 0;
    double refine_tol = 0.0;
    int64_t step = 0;
    int cur = 0;                       // which label buffer holds the current labels
    int64_t sweeps = 0, sm_calls = 0;
    int last_pass = -1;
    int tables_valid = 0;              // a sweep has drawn parameters since init/set_state
    Ws ws{};
    int32_t* c[2] = {nullptr, nullptr};
    uint8_t* cs[2] = {nullptr, nullptr};
    int64_t* tiles = nullptr;
    void* dbg = nullptr;
    int32_t dbg_cap = 0;
    int32_t dbg64 = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev;        // pairs (start, stop)
    std::vector<int> ev_stage;         // stage of each pair
    int n_timed = 0;
    int32_t* k_host = nullptr;         // pinned copy of K, refreshed after every call
    bool in_scratch = false;           // workspace and context live in the per-device static storage
    int since_layout = 0;              // sweeps since the cluster-sorted copy was last considered
    int64_t rs_ready_step = -1;        // step of the random split whose coins and halves the last sweep built
};

namespace {

dpmm_status set_device(dpmm_ctx* ctx)
{
    HIP_TRY(hipSetDevice(ctx->device));
    return DPMM_OK;
}

// Stage timing: while enabled, each stage of a sweep, split/merge call or
// empirical-Bayes step is bracketed by a pair of events on the stream.
struct StageTimer {
    dpmm_ctx* ctx;
    int pair = -1;
    StageTimer(dpmm_ctx* c, int stage) : ctx(c)
    {
        if (!ctx->timing || ctx->n_timed >= kMaxTimed) return;
        pair = ctx->n_timed++;
        ctx->ev_stage[pair] = stage;
        if (hipEventRecord(ctx->ev[2 * pair], ctx->stream) != hipSuccess) pair = -1;
    }
    ~StageTimer()
    {
        if (pair >= 0) hipEventRecord(ctx->ev[2 * pair + 1], ctx->stream);
    }
};

dpmm_status read_state(dpmm_ctx* ctx, DevState* out)
{
    HIP_TRY(hipMemcpyAsync(out, ctx->ws.st, sizeof(DevState), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DPMM_OK;
}

// queue a copy of the device K into the pinned hint (read by later launches)
dpmm_status refresh_k_hint(dpmm_ctx* ctx)
{
    if (!ctx->k_host) return DPMM_OK;
    HIP_TRY(hipMemcpyAsync(ctx->k_host, &ctx->ws.st->K, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    return DPMM_OK;
}

// Without the mapped hint (a context in static storage) launches are sized for
// k_max; the kernels loop over cluster groups either way.
int32_t k_hint(const dpmm_ctx* ctx)
{
    return ctx->k_host ? *reinterpret_cast<volatile int32_t*>(ctx->k_host) : ctx->k_max;
}

// statistics from the current labels, then compaction without touching
// flags; with split-BF16 the cluster-sorted copy is rebuilt from the labels
dpmm_status recompute_stats(dpmm_ctx* ctx)
{
    // no sweep has drawn these labels: no proposal term yet (all NaN); the
    // per-cluster sums of the term start at zero (each split pass clears
    // them again after use)
    if (ctx->ws.subdd) HIP_TRY(hipMemsetAsync(ctx->ws.subdd, 0xFF, 8 * (size_t)ctx->N, ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->ws.qsub, 0, sizeof(double) * (size_t)ctx->k_max, ctx->stream));
    launch_stats(ctx->ws, ctx->c[ctx->cur], ctx->cs[ctx->cur], ctx->stream);
    launch_compact(ctx->ws, 0, ctx->stream);
    launch_relabel(ctx->ws, ctx->c[ctx->cur], ctx->cs[ctx->cur], ctx->stream);
    if (ctx->precision == DPMM_SPLIT_BF16) launch_relayout(ctx->ws, ctx->c[ctx->cur], ctx->tiles, 1, ctx->stream);
    HIP_TRY(hipGetLastError());
    ctx->since_layout = 0;
    return DPMM_OK;
}

}  // namespace

extern "C" {

const char* dpmm_last_error(void) { return g_err; }

dpmm_status dpmm_workspace_size(const dpmm_csr* csr, const dpmm_params* params, size_t* bytes)
{
    dpmm_status s = check_args(csr, params);
    if (s != DPMM_OK) return s;
    if (!bytes) return fail(DPMM_ERR_ARG, "null bytes");
    *bytes = plan(csr->n_cells, csr->n_genes, csr->nnz, params->k_max, params->precision, params->flags).total;
    return DPMM_OK;
}

}  // extern "C"

namespace {

// dpmm_init, with the host context either allocated (static_slot == nullptr)
// or placed in a caller-provided slot, and the K hint either in mapped pinned
// host memory or, in the static slot's case, in a device word (hint_dev).
dpmm_status init_impl(const dpmm_csr* csr, const dpmm_params* params, void* workspace, size_t workspace_bytes,
                      void* stream, dpmm_ctx** out, dpmm_ctx* static_slot, int32_t* hint_dev)
{
    g_err[0] = 0;
    dpmm_status s = check_args(csr, params);
    if (s != DPMM_OK) return s;
    if (!out) return fail(DPMM_ERR_ARG, "null out");
    *out = nullptr;
    if (!workspace || ((uintptr_t)workspace & (kAlign - 1))) return fail(DPMM_ERR_ARG, "workspace must be 256-byte aligned");
    if (!csr->row_ptr || (csr->nnz > 0 && (!csr->col || !csr->val))) return fail(DPMM_ERR_ARG, "null CSR array");
    const Layout L = plan(csr->n_cells, csr->n_genes, csr->nnz, params->k_max, params->precision, params->flags);
    if (workspace_bytes < L.total)
        return fail(DPMM_ERR_NOMEM, "workspace of %zu bytes, %zu needed", workspace_bytes, L.total);

    dpmm_ctx* ctx = static_slot ? static_slot : new (std::nothrow) dpmm_ctx();
    if (!ctx) return fail(DPMM_ERR_NOMEM, "host allocation failed");
    ctx->in_scratch = static_slot != nullptr;
    auto release = [](dpmm_ctx* c) {
        if (c->in_scratch) *c = dpmm_ctx();
        else delete c;
    };
    hipError_t he = hipGetDevice(&ctx->device);
    if (he != hipSuccess) { release(ctx); return fail(DPMM_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(he)); }
    ctx->stream = (hipStream_t)stream;
    ctx->N = csr->n_cells;
    ctx->nnz = csr->nnz;
    ctx->G = csr->n_genes;
    ctx->k_max = params->k_max;
    ctx->precision = params->precision;
    ctx->refine_tol = params->refine_tol < 0.0 ? 0.0 : params->refine_tol;

    char* base = (char*)workspace;
    Ws& ws = ctx->ws;
    ws.N = csr->n_cells;
    ws.G = csr->n_genes;
    ws.k_max = params->k_max;
    ws.kpad = (params->k_max + 15) / 16 * 16;
    ws.Gpad = num_chunks(csr->n_genes) * kBlkGenes;
    ws.alpha = params->alpha;
    ws.seed = params->seed;
    ws.ent = (const uint32_t*)(base + L.ent);
    ws.roff = (const int64_t*)(base + L.roff);
    ws.st = (DevState*)(base + L.st);
    ws.reset = (uint8_t*)(base + L.reset);
    ws.nsub = (unsigned long long*)(base + L.nsub);
    ws.ssub = (unsigned long long*)(base + L.ssub);
    ws.beta = (double*)(base + L.beta);
    ws.lgbeta = (double*)(base + L.lgbeta);
    ws.lgrise = (double*)(base + L.lgrise);
    ws.flags = params->flags;
    ws.subdd = (params->flags & kFlagSplitQ) ? (double*)(base + L.subdd) : nullptr;
    ws.qsub = (double*)(base + L.qsub);
    const bool rsplit = (params->flags & kFlagRandomSplit) != 0;
    ws.rbits = rsplit ? (uint8_t*)(base + L.rbits) : nullptr;
    ws.rssub = rsplit ? (unsigned long long*)(base + L.rssub) : nullptr;
    ws.rnsub = rsplit ? (unsigned long long*)(base + L.rnsub) : nullptr;
    ws.logpi = (double*)(base + L.logpi);
    ws.lt64 = (double*)(base + L.lt64);
    ws.lc32 = (float*)(base + L.lc32);
    ws.ls32 = (float2*)(base + L.ls32);
    ws.lhi = (uint16_t*)(base + L.lhi);
    ws.llo = (uint16_t*)(base + L.llo);
    ws.refine = (uint32_t*)(base + L.refine);
    ws.perm = (int32_t*)(base + L.perm);
    ws.srow = (uint4*)(base + L.srow);
    ws.grp_cnt = (int32_t*)(base + L.grp_cnt);
    ws.grp_off = (int32_t*)(base + L.grp_off);
    ws.grp_cur = (int32_t*)(base + L.grp_cur);
    ws.nsub_prev = (unsigned long long*)(base + L.nsub_prev);
    ws.lay_kc = (int32_t*)(base + L.lay_kc);
    ws.lay_pbeg = (int32_t*)(base + L.lay_pbeg);
    ws.lay_pcnt = (int32_t*)(base + L.lay_pcnt);
    ws.lay_cell = (int32_t*)(base + L.lay_cell);
    ws.lay_doff = (int64_t*)(base + L.lay_doff);
    ws.lay_toff = (int64_t*)(base + L.lay_toff);
    ws.lay_dense = (uint8_t*)(base + L.lay_dense);
    ws.lay_tail = (uint32_t*)(base + L.lay_tail);
    ws.lay_nnz = (uint16_t*)(base + L.lay_nnz);
    ws.lay_hcnt = (uint8_t*)(base + L.lay_hcnt);
    ws.lay_bh = (uint8_t*)(base + L.lay_bh);
    ws.lay_rank = (uint16_t*)(base + L.lay_rank);
    ws.lay_gene = (uint16_t*)(base + L.lay_gene);
    ws.lay_bhi = (uint16_t*)(base + L.lay_bhi);
    ws.lay_blo = (uint16_t*)(base + L.lay_blo);
    ws.lay_lim = (uint64_t*)(base + L.lay_lim);
    ws.lay_dE = (int32_t*)(base + L.lay_dE);
    ws.lay_dS = (int32_t*)(base + L.lay_dS);
    ws.lay_dfull = (double*)(base + L.lay_dfull);
    ws.lay_sw = (double*)(base + L.lay_sw);
    ws.lay_part = (uint32_t*)(base + L.lay_part);
    ws.mov = (uint32_t*)(base + L.mov);
    ws.lay_pw = params->precision == DPMM_SPLIT_BF16 ? lay_hist_words(params->flags) : 0;
    ws.lay_bbeg = (int32_t*)(base + L.lay_bbeg);
    ws.lay_sbeg = (int32_t*)(base + L.lay_sbeg);
    ws.nblk_cap = params->precision == DPMM_SPLIT_BF16 ? lay_blocks(csr->n_cells, params->k_max) : 0;
    ws.lay_cols = lay_cols(params->k_max);
    ws.relab_c = (int32_t*)(base + L.relab_c);
    ws.relab_s = (uint8_t*)(base + L.relab_s);
    ws.sm_logr = (double*)(base + L.sm_logr);
    ws.sm_acc = (uint8_t*)(base + L.sm_acc);
    ws.mkey = (unsigned long long*)(base + L.mkey);
    ws.mlist = (int32_t*)(base + L.mlist);
    ws.dm_k = (double*)(base + L.dm_k);
    ws.eb_tmp = (double*)(base + L.eb_tmp);
    ws.rd_part = (double2*)(base + L.rd_part);
    ws.sm_part = (SmPart*)(base + L.sm_part);
    ctx->c[0] = (int32_t*)(base + L.c0);
    ctx->c[1] = (int32_t*)(base + L.c1);
    ctx->cs[0] = (uint8_t*)(base + L.cs0);
    ctx->cs[1] = (uint8_t*)(base + L.cs1);
    ctx->tiles = (int64_t*)(base + L.tiles);

    auto cleanup = [&](dpmm_status st) {
        if (ctx->k_host) hipHostFree(ctx->k_host);
        release(ctx);
        return st;
    };
    if (hint_dev) {
        ws.k_hint = hint_dev;
    } else {
        he = hipHostMalloc((void**)&ctx->k_host, sizeof(int32_t), hipHostMallocMapped);
        if (he != hipSuccess) { ctx->k_host = nullptr; return cleanup(fail(DPMM_ERR_HIP, "hipHostMalloc: %s", hipGetErrorString(he))); }
        *ctx->k_host = params->k_init;
        he = hipHostGetDevicePointer((void**)&ws.k_hint, ctx->k_host, 0);
        if (he != hipSuccess) return cleanup(fail(DPMM_ERR_HIP, "hipHostGetDevicePointer: %s", hipGetErrorString(he)));
    }
    if (params->precision == DPMM_SPLIT_BF16) {
        he = configure_assign_bf16();
        if (he == hipSuccess) he = configure_layout();
        if (he != hipSuccess) return cleanup(fail(DPMM_ERR_HIP, "kernel attributes: %s", hipGetErrorString(he)));
    }
    he = sub_stats_cells(ws.N, ws.G, &ws.sub_cells);
    if (he != hipSuccess) return cleanup(fail(DPMM_ERR_HIP, "occupancy query: %s", hipGetErrorString(he)));
    he = hipMemsetAsync(ws.st, 0, sizeof(DevState), ctx->stream);
    if (he == hipSuccess) he = hipMemsetAsync(ws.lc32, 0, L.ls32 - L.lc32, ctx->stream);
    if (he == hipSuccess) he = hipMemsetAsync(ws.lhi, 0, L.refine - L.lhi, ctx->stream);
    if (he != hipSuccess) return cleanup(fail(DPMM_ERR_HIP, "hipMemsetAsync: %s", hipGetErrorString(he)));
    launch_pack(csr->row_ptr, csr->col, csr->val, csr->n_cells, csr->n_genes, csr->nnz, (int64_t*)ws.roff,
                ctx->tiles, (uint32_t*)ws.ent, ws.st, ctx->stream);
    if (params->beta_per_gene)
        he = hipMemcpyAsync(ws.beta, params->beta_per_gene, 8 * (size_t)ws.G, hipMemcpyDeviceToDevice, ctx->stream);
    else
        launch_fill(ws.beta, ws.G, params->beta, ctx->stream);
    if (he != hipSuccess) return cleanup(fail(DPMM_ERR_HIP, "beta copy: %s", hipGetErrorString(he)));
    launch_lgamma_beta(ws, ctx->stream);
    launch_init_labels(ws, params->k_init, ctx->c[0], ctx->cs[0], ctx->stream);
    he = hipGetLastError();
    if (he != hipSuccess) return cleanup(fail(DPMM_ERR_HIP, "init launch: %s", hipGetErrorString(he)));
    DevState dst;
    he = hipMemcpyAsync(&dst, ws.st, sizeof(DevState), hipMemcpyDeviceToHost, ctx->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
    if (he != hipSuccess) return cleanup(fail(DPMM_ERR_HIP, "init sync: %s", hipGetErrorString(he)));
    if (dst.data_error) return cleanup(fail(DPMM_ERR_DATA, "CSR validation failed on %d rows", dst.data_error));
    // the input's row_ptr[N] must equal nnz
    int64_t last = 0;
    he = hipMemcpy(&last, csr->row_ptr + csr->n_cells, sizeof(int64_t), hipMemcpyDeviceToHost);
    if (he != hipSuccess) return cleanup(fail(DPMM_ERR_HIP, "row_ptr read: %s", hipGetErrorString(he)));
    if (last != csr->nnz) return cleanup(fail(DPMM_ERR_DATA, "row_ptr[N] = %lld differs from nnz = %lld",
                                              (long long)last, (long long)csr->nnz));
    s = recompute_stats(ctx);
    if (s == DPMM_OK) s = refresh_k_hint(ctx);
    if (s != DPMM_OK) return cleanup(s);
    he = hipStreamSynchronize(ctx->stream);
    if (he != hipSuccess) return cleanup(fail(DPMM_ERR_HIP, "init stats: %s", hipGetErrorString(he)));
    *out = ctx;
    return DPMM_OK;
}

// ---------------------------------------------------------------------------
// Static storage for dpmm_init_static: a workspace of kScratchBytes per device
// (the last 256 bytes hold the K hint) and one host context slot per device.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr size_t kScratchHint = 256;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices];          // device address of scratch, per device
bool g_scratch_busy[kMaxDevices];          // a context holds the device's storage
dpmm_ctx g_scratch_ctx[kMaxDevices];

}  // namespace

extern "C" {

dpmm_status dpmm_init(const dpmm_csr* csr, const dpmm_params* params, void* workspace, size_t workspace_bytes,
                      void* stream, dpmm_ctx** out)
{
    return init_impl(csr, params, workspace, workspace_bytes, stream, out, nullptr, nullptr);
}

dpmm_status dpmm_init_static(const dpmm_csr* csr, const dpmm_params* params, void* stream, dpmm_ctx** out)
{
    g_err[0] = 0;
    dpmm_status s = check_args(csr, params);
    if (s != DPMM_OK) return s;
    if (!out) return fail(DPMM_ERR_ARG, "null out");
    *out = nullptr;
    const size_t need = plan(csr->n_cells, csr->n_genes, csr->nnz, params->k_max, params->precision, params->flags).total;
    if (need > kScratchBytes - kScratchHint)
        return fail(DPMM_ERR_NOMEM, "dpmm_init_static: %zu bytes of workspace needed, the static workspace holds %zu",
                    need, kScratchBytes - kScratchHint);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DPMM_ERR_UNSUPPORTED, "device %d beyond the static slots", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_busy[dev]) return fail(DPMM_ERR_STATE, "the static workspace of device %d is held by a context", dev);
    if (!g_scratch_ptr[dev]) {
        // the symbol's address on this device (each device holds its own copy)
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(DPMM_ERR_HIP, "hipGetSymbolAddress returned no address");
        g_scratch_ptr[dev] = p;
    }
    char* base = static_cast<char*>(g_scratch_ptr[dev]);
    int32_t* hint = reinterpret_cast<int32_t*>(base + kScratchBytes - kScratchHint);
    s = init_impl(csr, params, base, kScratchBytes - kScratchHint, stream, out, &g_scratch_ctx[dev], hint);
    if (s == DPMM_OK) g_scratch_busy[dev] = true;
    return s;
}


dpmm_status dpmm_destroy(dpmm_ctx* ctx)
{
    if (!ctx) return fail(DPMM_ERR_ARG, "null ctx");
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->ev) hipEventDestroy(e);
    if (ctx->k_host) hipHostFree(ctx->k_host);
    if (ctx->in_scratch) {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        const int dev = ctx->device;
        *ctx = dpmm_ctx();
        if (dev >= 0 && dev < kMaxDevices) g_scratch_busy[dev] = false;
    } else {
        delete ctx;
    }
    return DPMM_OK;
}

// The move of the split/merge call at `step`: 0 split into the sub-clusters,
// 1 merges, 2 random splits (only with DPMM_FLAG_RANDOM_SPLIT, the three then
// equally likely).  The chain coin depends only on (seed, step).
static int chain_pass(const dpmm_ctx* ctx, uint32_t step)
{
    const Words w = philox(ctx->ws.seed, 0u, 0u, step, kChain, 0u);
    const double coin = unit52(w.w[0], w.w[1]);
    if (ctx->ws.flags & kFlagRandomSplit) return coin < 1.0 / 3.0 ? 0 : (coin < 2.0 / 3.0 ? 2 : 1);
    return coin < 0.5 ? 0 : 1;
}

dpmm_status dpmm_sweep(dpmm_ctx* ctx, int32_t n_sweeps)
{
    if (!ctx) return fail(DPMM_ERR_ARG, "null ctx");
    if (n_sweeps < 0) return fail(DPMM_ERR_ARG, "n_sweeps must be >= 0");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    const Ws& ws = ctx->ws;
    for (int32_t n = 0; n < n_sweeps; ++n) {
        const int nxt = 1 - ctx->cur;
        const uint32_t step = (uint32_t)ctx->step;
        if (ctx->precision == DPMM_SPLIT_BF16 && ++ctx->since_layout >= kRelayoutEvery) {
            // rebuild the cluster-sorted copy if the partition changed
            // structurally (a deterministic, device-side decision)
            StageTimer st(ctx, DPMM_STAGE_LAYOUT);
            launch_relayout(ws, ctx->c[ctx->cur], ctx->tiles, 0, ctx->stream);
            ctx->since_layout = 0;
        }
        // a random split next: its coins and coin halves come with this pass
        const bool rsplit = n + 1 == n_sweeps && ws.rssub && chain_pass(ctx, step + 1) == 2;
        {
            StageTimer st(ctx, DPMM_STAGE_REDRAW);
            if (ws.flags & kFlagNewCluster) launch_extend(ws, ctx->stream);
            // (also empties the re-score queue, and clears the coin halves for rsplit)
            const int kg = k_hint(ctx) + ((ws.flags & kFlagNewCluster) ? 1 : 0);   // sizes grids
            launch_redraw(ws, step, ctx->precision == DPMM_SPLIT_BF16, rsplit, kg, ctx->stream);
            if (ctx->precision == DPMM_SPLIT_BF16) launch_lay_btab(ws, kg, ctx->stream);
        }
        AssignArgs a{};
        a.c_old = ctx->c[ctx->cur];
        a.cs_old = ctx->cs[ctx->cur];
        a.c_new = ctx->c[nxt];
        a.cs_new = ctx->cs[nxt];
        a.step = step;
        a.dbg = ctx->dbg;
        a.dbg_stride = ctx->dbg_cap + 2;
        a.dbg64 = ctx->dbg64;
        a.refine = ctx->precision != DPMM_FP64;
        a.refine_tol = (float)ctx->refine_tol;
        a.k_hint = k_hint(ctx);
        SubArgs sa{};
        sa.c_old = ctx->c[ctx->cur];
        sa.cs_old = ctx->cs[ctx->cur];
        sa.c_new = ctx->c[nxt];
        sa.cs_new = ctx->cs[nxt];
        sa.step = step;
        sa.dbg = ctx->dbg;
        sa.dbg_stride = ctx->dbg_cap + 2;
        sa.dbg64 = ctx->dbg64;
        if (rsplit) {
            sa.rsplit = 1;
            sa.rs_step = step + 1;
        }
        ctx->rs_ready_step = sa.rsplit ? (int64_t)ctx->step + 1 : -1;
        // split-BF16 without a score dump: the sub-cluster pass of the cells
        // that keep their block's cluster runs inside the cluster draw
        const bool fused = ctx->precision == DPMM_SPLIT_BF16 && !ctx->dbg;
        {
            StageTimer st(ctx, DPMM_STAGE_ASSIGN);
            if (ctx->precision == DPMM_FP64) launch_assign_fp64(ws, a, ctx->stream);
            else if (ctx->precision == DPMM_FP32) launch_assign_fp32(ws, a, ctx->stream);
            else launch_assign_bf16(ws, a, fused ? &sa : nullptr, ctx->stream);
        }
        if (a.refine && !fused) {      // (the fused pass re-scores in its queue kernel)
            StageTimer st(ctx, DPMM_STAGE_REFINE);
            launch_refine(ws, a, ctx->stream);
        }
        {
            StageTimer st(ctx, DPMM_STAGE_SUBCLUSTER);
            if (fused) launch_lay_sub_rest(ws, sa, ctx->stream);
            else if (ctx->precision == DPMM_SPLIT_BF16) launch_lay_sub(ws, sa, ctx->stream);
            else launch_sub_stats(ws, sa, ctx->stream);
        }
        {
            StageTimer st(ctx, DPMM_STAGE_COMPACT);
            launch_compact(ws, 1, ctx->stream);
            launch_relabel(ws, ctx->c[nxt], ctx->cs[nxt], ctx->stream);
        }
        HIP_TRY(hipGetLastError());     // (k_compact has written the K hint)
        ctx->cur = nxt;
        ctx->step += 1;
        ctx->sweeps += 1;
        ctx->tables_valid = 1;
    }
    return DPMM_OK;
}

dpmm_status dpmm_split_merge(dpmm_ctx* ctx)
{
    if (!ctx) return fail(DPMM_ERR_ARG, "null ctx");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    const uint32_t step = (uint32_t)ctx->step;
    const int pass = chain_pass(ctx, step);    // drawn here, without a sync
    const bool ready = ctx->rs_ready_step == ctx->step;
    ctx->rs_ready_step = -1;
    StageTimer st(ctx, DPMM_STAGE_SPLIT_MERGE);
    const int kg = k_hint(ctx);     // sizes the grids (any K is covered)
    if (pass == 1) {
        launch_merge_ratios(ctx->ws, kg, ctx->stream);
        launch_sm_decide(ctx->ws, 1, step, ctx->stream);
    } else if (pass == 0) {
        launch_split_ratios(ctx->ws, ctx->c[ctx->cur], ctx->cs[ctx->cur], kg, ctx->stream);
        launch_sm_decide(ctx->ws, 0, step, ctx->stream);
    } else {
        launch_random_split(ctx->ws, ctx->c[ctx->cur], ctx->cs[ctx->cur], step, ready, kg, ctx->stream);
    }
    launch_relabel(ctx->ws, ctx->c[ctx->cur], ctx->cs[ctx->cur], ctx->stream);
    HIP_TRY(hipGetLastError());     // (k_sm_decide has written the K hint)
    ctx->last_pass = pass;
    ctx->step += 1;
    ctx->sm_calls += 1;
    return DPMM_OK;
}

dpmm_status dpmm_eb_update(dpmm_ctx* ctx)
{
    if (!ctx) return fail(DPMM_ERR_ARG, "null ctx");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    {
        StageTimer st(ctx, DPMM_STAGE_EB);
        launch_eb_update(ctx->ws, ctx->stream);
    }
    HIP_TRY(hipGetLastError());
    return DPMM_OK;
}

dpmm_status dpmm_stats(dpmm_ctx* ctx, dpmm_stats_out* out, int64_t* nsub_host, int64_t* ssub_dev)
{
    if (!ctx || !out) return fail(DPMM_ERR_ARG, "null argument");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    launch_log_joint(ctx->ws, ctx->stream);
    HIP_TRY(hipGetLastError());
    DevState d;
    s = read_state(ctx, &d);
    if (s != DPMM_OK) return s;
    memset(out, 0, sizeof(*out));
    out->step = ctx->step;
    out->K = d.K;
    out->last_pass = ctx->last_pass;
    out->sweeps = ctx->sweeps;
    out->sm_calls = ctx->sm_calls;
    out->splits_proposed = (int64_t)d.counters[kCntSplitsProposed];
    out->splits_accepted = (int64_t)d.counters[kCntSplitsAccepted];
    out->merges_proposed = (int64_t)d.counters[kCntMergesProposed];
    out->merges_accepted = (int64_t)d.counters[kCntMergesAccepted];
    out->kmax_skips = (int64_t)d.counters[kCntKmaxSkips];
    out->refined = (int64_t)d.counters[kCntRefined];
    out->gamma_caps = (int64_t)d.counters[kCntGammaCaps];
    out->evals = (int64_t)d.counters[kCntEvals];
    out->near_tie = (int64_t)d.counters[kCntNearTie];
    out->log_joint = d.log_joint;
    if (nsub_host)
        HIP_TRY(hipMemcpy(nsub_host, ctx->ws.nsub, 16 * (size_t)d.K, hipMemcpyDeviceToHost));
    if (ssub_dev)
        HIP_TRY(hipMemcpyAsync(ssub_dev, ctx->ws.ssub, 16 * (size_t)d.K * (size_t)ctx->G, hipMemcpyDeviceToDevice,
                               ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DPMM_OK;
}

dpmm_status dpmm_get_labels(dpmm_ctx* ctx, int32_t* c_dev, uint8_t* cs_dev)
{
    if (!ctx || !c_dev || !cs_dev) return fail(DPMM_ERR_ARG, "null argument");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    HIP_TRY(hipMemcpyAsync(c_dev, ctx->c[ctx->cur], 4 * (size_t)ctx->N, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(cs_dev, ctx->cs[ctx->cur], (size_t)ctx->N, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DPMM_OK;
}

dpmm_status dpmm_set_state(dpmm_ctx* ctx, int64_t step, int32_t K, const int32_t* c_dev, const uint8_t* cs_dev,
                           const uint8_t* reset_host)
{
    if (!ctx || !c_dev || !cs_dev || !reset_host) return fail(DPMM_ERR_ARG, "null argument");
    if (K < 1 || K > ctx->k_max) return fail(DPMM_ERR_ARG, "K must be in [1, k_max]");
    if (step < 0 || step > 0xFFFFFFFFll) return fail(DPMM_ERR_ARG, "step must be in [0, 2^32)");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    const Ws& ws = ctx->ws;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->c[0], c_dev, 4 * (size_t)ctx->N, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->cs[0], cs_dev, (size_t)ctx->N, hipMemcpyDeviceToDevice, ctx->stream));
    std::vector<uint8_t> flags((size_t)ctx->k_max, 0);
    for (int k = 0; k < K; ++k) flags[k] = reset_host[k] ? 1 : 0;
    HIP_TRY(hipMemcpyAsync(ws.reset, flags.data(), (size_t)ctx->k_max, hipMemcpyHostToDevice, ctx->stream));
    DevState d;
    memset(&d, 0, sizeof(d));
    d.K = K;
    HIP_TRY(hipMemcpyAsync(ws.st, &d, sizeof(d), hipMemcpyHostToDevice, ctx->stream));
    ctx->cur = 0;
    launch_check_labels(ws, ctx->c[0], ctx->cs[0], K, ctx->stream);
    DevState chk;
    s = read_state(ctx, &chk);
    if (s != DPMM_OK) return s;
    if (chk.data_error) {
        HIP_TRY(hipMemsetAsync(&ws.st->data_error, 0, sizeof(int32_t), ctx->stream));
        return fail(DPMM_ERR_ARG, "%d labels out of range", chk.data_error);
    }
    s = recompute_stats(ctx);
    if (s == DPMM_OK) s = refresh_k_hint(ctx);
    if (s != DPMM_OK) return s;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->step = step;
    ctx->sweeps = ctx->sm_calls = 0;
    ctx->last_pass = -1;
    ctx->rs_ready_step = -1;
    return DPMM_OK;
}

dpmm_status dpmm_get_reset_flags(dpmm_ctx* ctx, uint8_t* reset_host)
{
    if (!ctx || !reset_host) return fail(DPMM_ERR_ARG, "null argument");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    DevState d;
    s = read_state(ctx, &d);
    if (s != DPMM_OK) return s;
    HIP_TRY(hipMemcpy(reset_host, ctx->ws.reset, (size_t)d.K, hipMemcpyDeviceToHost));
    return DPMM_OK;
}

dpmm_status dpmm_get_params(dpmm_ctx* ctx, double* logpi_dev, double* logtheta_dev)
{
    if (!ctx) return fail(DPMM_ERR_ARG, "null ctx");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    if (logpi_dev)
        HIP_TRY(hipMemcpyAsync(logpi_dev, ctx->ws.logpi, 8 * (size_t)ctx->k_max, hipMemcpyDeviceToDevice, ctx->stream));
    if (logtheta_dev)
        HIP_TRY(hipMemcpyAsync(logtheta_dev, ctx->ws.lt64, 24 * (size_t)ctx->k_max * (size_t)ctx->G,
                               hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DPMM_OK;
}

dpmm_status dpmm_get_beta(dpmm_ctx* ctx, double* beta_dev)
{
    if (!ctx || !beta_dev) return fail(DPMM_ERR_ARG, "null argument");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    HIP_TRY(hipMemcpyAsync(beta_dev, ctx->ws.beta, 8 * (size_t)ctx->G, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DPMM_OK;
}

dpmm_status dpmm_set_beta(dpmm_ctx* ctx, const double* beta_dev)
{
    if (!ctx || !beta_dev) return fail(DPMM_ERR_ARG, "null argument");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    HIP_TRY(hipMemcpyAsync(ctx->ws.beta, beta_dev, 8 * (size_t)ctx->G, hipMemcpyDeviceToDevice, ctx->stream));
    launch_lgamma_beta(ctx->ws, ctx->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DPMM_OK;
}

dpmm_status dpmm_get_hastings(dpmm_ctx* ctx, int32_t* pass, int32_t* n, double* logr_host, uint8_t* accept_host)
{
    if (!ctx || !pass || !n) return fail(DPMM_ERR_ARG, "null argument");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    DevState d;
    s = read_state(ctx, &d);
    if (s != DPMM_OK) return s;
    *pass = ctx->last_pass;
    *n = ctx->last_pass < 0 ? 0 : d.sm_n;
    if (*n > 0 && logr_host) HIP_TRY(hipMemcpy(logr_host, ctx->ws.sm_logr, 8 * (size_t)*n, hipMemcpyDeviceToHost));
    if (*n > 0 && accept_host) HIP_TRY(hipMemcpy(accept_host, ctx->ws.sm_acc, (size_t)*n, hipMemcpyDeviceToHost));
    return DPMM_OK;
}

dpmm_status dpmm_set_debug_scores(dpmm_ctx* ctx, void* scores_dev, int32_t k_cap, int32_t fp64)
{
    if (!ctx) return fail(DPMM_ERR_ARG, "null ctx");
    if (scores_dev && (k_cap < 1 || k_cap > ctx->k_max)) return fail(DPMM_ERR_ARG, "k_cap must be in [1, k_max]");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->dbg = scores_dev;
    ctx->dbg_cap = scores_dev ? k_cap : 0;
    ctx->dbg64 = fp64 ? 1 : 0;
    return DPMM_OK;
}

dpmm_status dpmm_dump_scores(dpmm_ctx* ctx, const int32_t* cells_dev, int32_t m, double* out_dev)
{
    if (!ctx) return fail(DPMM_ERR_ARG, "null ctx");
    if (m < 0) return fail(DPMM_ERR_ARG, "m must be >= 0");
    if (m > 0 && (!cells_dev || !out_dev)) return fail(DPMM_ERR_ARG, "null argument");
    if (!ctx->tables_valid) return fail(DPMM_ERR_STATE, "no sweep has drawn parameters yet");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    if (m > 0) launch_dump_scores(ctx->ws, ctx->c[ctx->cur], cells_dev, m, out_dev, ctx->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DPMM_OK;
}

dpmm_status dpmm_get_split_tables(dpmm_ctx* ctx, uint16_t* hi_dev, uint16_t* lo_dev)
{
    if (!ctx || !hi_dev || !lo_dev) return fail(DPMM_ERR_ARG, "null argument");
    if (ctx->precision != DPMM_SPLIT_BF16) return fail(DPMM_ERR_STATE, "context is not split-BF16");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    DevState d;
    s = read_state(ctx, &d);
    if (s != DPMM_OK) return s;
    // cluster-major [k][Gpad] -> K x G
    for (int k = 0; k < d.K; ++k) {
        HIP_TRY(hipMemcpyAsync(hi_dev + (size_t)k * ctx->G, ctx->ws.lhi + (size_t)k * ctx->ws.Gpad, 2 * (size_t)ctx->G,
                               hipMemcpyDeviceToDevice, ctx->stream));
        HIP_TRY(hipMemcpyAsync(lo_dev + (size_t)k * ctx->G, ctx->ws.llo + (size_t)k * ctx->ws.Gpad, 2 * (size_t)ctx->G,
                               hipMemcpyDeviceToDevice, ctx->stream));
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return DPMM_OK;
}

dpmm_status dpmm_timing_enable(dpmm_ctx* ctx, int32_t enable)
{
    if (!ctx) return fail(DPMM_ERR_ARG, "null ctx");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    if (enable && ctx->ev.empty()) {
        ctx->ev.resize(2 * kMaxTimed);
        ctx->ev_stage.assign(kMaxTimed, 0);
        for (auto& e : ctx->ev) HIP_TRY(hipEventCreate(&e));
    }
    ctx->timing = enable != 0;
    return DPMM_OK;
}

dpmm_status dpmm_timing_stages(dpmm_ctx* ctx, double* stage_ms, int64_t* stage_count)
{
    if (!ctx || !stage_ms || !stage_count) return fail(DPMM_ERR_ARG, "null argument");
    dpmm_status s = set_device(ctx);
    if (s != DPMM_OK) return s;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < DPMM_NUM_STAGES; ++q) {
        stage_ms[q] = 0.0;
        stage_count[q] = 0;
    }
    for (int q = 0; q < ctx->n_timed; ++q) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[2 * q], ctx->ev[2 * q + 1]));
        stage_ms[ctx->ev_stage[q]] += ms;
        stage_count[ctx->ev_stage[q]] += 1;
    }
    ctx->n_timed = 0;
    return DPMM_OK;
}

dpmm_status dpmm_timing_read(dpmm_ctx* ctx, double* total_ms, int64_t* launches)
{
    if (!ctx || !total_ms || !launches) return fail(DPMM_ERR_ARG, "null argument");
    double ms[DPMM_NUM_STAGES];
    int64_t cnt[DPMM_NUM_STAGES];
    dpmm_status s = dpmm_timing_stages(ctx, ms, cnt);
    if (s != DPMM_OK) return s;
    *total_ms = ms[DPMM_STAGE_ASSIGN];
    *launches = cnt[DPMM_STAGE_ASSIGN];
    return DPMM_OK;
}

dpmm_status dpmm_gene_moments(const dpmm_csr* csr, uint64_t* sum_dev, uint64_t* sumsq_dev, void* stream)
{
    if (!csr || !sum_dev || !sumsq_dev) return fail(DPMM_ERR_ARG, "null argument");
    if (csr->n_genes < 1 || csr->n_genes > 65535) return fail(DPMM_ERR_ARG, "n_genes must be in [1, 65535]");
    if (csr->nnz < 0 || (csr->nnz > 0 && (!csr->col || !csr->val))) return fail(DPMM_ERR_ARG, "bad entries");
    launch_gene_moments(csr->col, csr->val, csr->nnz, csr->n_genes, reinterpret_cast<unsigned long long*>(sum_dev),
                        reinterpret_cast<unsigned long long*>(sumsq_dev), (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return DPMM_OK;
}

dpmm_status dpmm_top_genes(const uint64_t* sum_dev, const uint64_t* sumsq_dev, int32_t n_genes, int64_t n_cells,
                           int32_t k, int32_t* map_dev, double* std_dev, void* stream)
{
    if (!sum_dev || !sumsq_dev || !map_dev) return fail(DPMM_ERR_ARG, "null argument");
    if (n_genes < 1 || n_genes > 65535) return fail(DPMM_ERR_ARG, "n_genes must be in [1, 65535]");
    if (n_cells < 1 || n_cells >= (1ll << 30)) return fail(DPMM_ERR_ARG, "n_cells must be in [1, 2^30)");
    if (k < 0) return fail(DPMM_ERR_ARG, "k must be >= 0");
    launch_top_genes(reinterpret_cast<const unsigned long long*>(sum_dev),
                     reinterpret_cast<const unsigned long long*>(sumsq_dev), n_genes, n_cells, k, map_dev, std_dev,
                     (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return DPMM_OK;
}

dpmm_status dpmm_filter_genes(const dpmm_csr* csr, const int32_t* map_dev, int64_t* row_ptr_out, int32_t* col_out,
                              int32_t* val_out, int64_t* nnz_out, void* stream)
{
    if (!csr || !map_dev || !row_ptr_out) return fail(DPMM_ERR_ARG, "null argument");
    if (csr->n_cells < 1 || csr->n_cells >= (1ll << 30)) return fail(DPMM_ERR_ARG, "n_cells must be in [1, 2^30)");
    if (csr->n_genes < 1 || csr->n_genes > 65535) return fail(DPMM_ERR_ARG, "n_genes must be in [1, 65535]");
    if (!csr->row_ptr || (csr->nnz > 0 && (!csr->col || !csr->val))) return fail(DPMM_ERR_ARG, "bad CSR");
    const hipStream_t s = (hipStream_t)stream;
    if (!col_out) {
        if (!nnz_out) return fail(DPMM_ERR_ARG, "nnz_out is needed by the first call");
        launch_filter_count(csr->row_ptr, csr->col, csr->n_cells, csr->n_genes, map_dev, row_ptr_out, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(nnz_out, row_ptr_out + csr->n_cells, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return DPMM_OK;
    }
    if (!val_out) return fail(DPMM_ERR_ARG, "null val_out");
    launch_filter_fill(csr->row_ptr, csr->col, csr->val, csr->n_cells, csr->n_genes, map_dev, row_ptr_out, col_out,
                       val_out, s);
    HIP_TRY(hipGetLastError());
    return DPMM_OK;
}

dpmm_status dpmm_dm_logmarginal(const int64_t* sv, int32_t J, int32_t G, const double* beta, double* out, void* stream)
{
    if (J < 0 || G < 1) return fail(DPMM_ERR_ARG, "J must be >= 0 and G >= 1");
    if (J == 0) return DPMM_OK;
    if (!sv || !beta || !out) return fail(DPMM_ERR_ARG, "null argument");
    launch_dm_logmarginal(sv, J, G, beta, out, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return DPMM_OK;
}

dpmm_status dpmm_dm_grad(const int64_t* sv, int32_t J, int32_t G, const double* beta, const double* g,
                         double* grad_beta, void* stream)
{
    if (J < 0 || G < 1) return fail(DPMM_ERR_ARG, "J must be >= 0 and G >= 1");
    if (!beta || !grad_beta || (J > 0 && (!sv || !g))) return fail(DPMM_ERR_ARG, "null argument");
    launch_dm_grad(sv, J, G, beta, g, grad_beta, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return DPMM_OK;
}

}  // extern "C"
