// kernels.hpp -- host-side launchers of the libdpmm kernels (all enqueue on
// the given stream and return immediately).
#pragma once

#include "dpmm_common.hpp"

namespace dpmm {

// bookkeeping.hip
void launch_zero(void* p, size_t bytes, hipStream_t s);   // bytes: a multiple of 4
// gate (device, may be null): the kernels do nothing unless *gate != 0
void launch_exclusive_scan(int64_t* v, int64_t n, int64_t* tile_sums, hipStream_t s, const int32_t* gate = nullptr);
void launch_pack(const int64_t* row_ptr, const int32_t* col, const int32_t* val, int64_t N, int32_t G, int64_t nnz,
                 int64_t* roff, int64_t* tile_sums, uint32_t* ent, DevState* st, hipStream_t s);
void launch_init_labels(const Ws& ws, int32_t k_init, int32_t* c, uint8_t* cs, hipStream_t s);
void launch_stats(const Ws& ws, const int32_t* c, const uint8_t* cs, hipStream_t s);
// c_prev (by cluster only, may be null): the labels before the sweep, whose
// membership of the cell's new cluster goes into the top bits of srow.w
void launch_sort(const Ws& ws, const int32_t* c, const uint8_t* cs, int by_cluster, hipStream_t s,
                 bool counts_cleared = false, const int32_t* c_prev = nullptr, const int32_t* gate = nullptr);

// layout.hip
// rebuild the cluster-sorted copy from labels c (force: unconditionally; else
// only when the partition changed structurally since the last build)
void launch_relayout(const Ws& ws, const int32_t* c, int64_t* tile_sums, int force, hipStream_t s);
void launch_lay_btab(const Ws& ws, int k_guess, hipStream_t s);   // k_guess: a recent K (sizes the grid)    // permuted hi/lo tables, after each redraw
hipError_t configure_layout();

// bookkeeping.hip
void launch_extend(const Ws& ws, hipStream_t s);
void launch_top_genes(const unsigned long long* sum, const unsigned long long* sumsq, int32_t G, int64_t N, int32_t k,
                      int32_t* map, double* std_out, hipStream_t s);
void launch_gene_moments(const int32_t* col, const int32_t* val, int64_t nnz, int32_t G, unsigned long long* sum,
                         unsigned long long* sumsq, hipStream_t s);
void launch_filter_count(const int64_t* row_ptr, const int32_t* col, int64_t N, int32_t G, const int32_t* map,
                         int64_t* out_ptr, hipStream_t s);
void launch_filter_fill(const int64_t* row_ptr, const int32_t* col, const int32_t* val, int64_t N, int32_t G,
                        const int32_t* map, const int64_t* out_ptr, int32_t* col_out, int32_t* val_out, hipStream_t s);

// substats.hip
struct SubArgs {
    const int32_t* c_old;
    const uint8_t* cs_old;
    int32_t* c_new;       // (written by the queue kernel for a re-scored cell)
    uint8_t* cs_new;
    uint32_t step;
    void* dbg;            // optional score dump (FP32, or FP64 when dbg64), row stride dbg_stride
    int32_t dbg_stride;
    int32_t dbg64;
    int32_t rsplit;       // also draw the coins of the random split at step rs_step and
    uint32_t rs_step;     // accumulate the statistics of the coin halves (rbits, rssub, rnsub)
};
void launch_sub_stats(const Ws& ws, const SubArgs& a, hipStream_t s);
// laysub.hip (split-BF16 sweeps, over the cluster-sorted copy)
void launch_lay_sub(const Ws& ws, const SubArgs& a, hipStream_t s);
// the rest of that pass (also after its fused form in launch_assign_bf16):
// the queued cells (those flagged kRefineCluster re-scored in FP64 first) and
// the sums of the block histograms, in one launch
void launch_lay_sub_rest(const Ws& ws, const SubArgs& a, hipStream_t s);
hipError_t sub_stats_cells(int64_t N, int G, int32_t* cells);
void launch_compact(const Ws& ws, int after_sweep, hipStream_t s);
void launch_relabel(const Ws& ws, int32_t* c, uint8_t* cs, hipStream_t s);
void launch_check_labels(const Ws& ws, const int32_t* c, const uint8_t* cs, int32_t K, hipStream_t s);

// redraw.hip
// zero_rs: also clear rssub / rnsub (a random split follows the sweep);
// k_guess: a recent K of the sweep (sizes the grid; any K is covered)
void launch_redraw(const Ws& ws, uint32_t step, int write_split, int zero_rs, int k_guess, hipStream_t s);

// assign.hip
struct AssignArgs {
    const int32_t* c_old;
    const uint8_t* cs_old;
    int32_t* c_new;
    uint8_t* cs_new;
    uint32_t step;
    void* dbg;            // optional score dump (FP32, or FP64 when dbg64), row stride dbg_stride
    int32_t dbg_stride;
    int32_t dbg64;
    int32_t refine;       // queue uncertain decisions for the FP64 re-score
    float refine_tol;     // extra relative-margin threshold (0: bound only)
    int32_t k_hint;       // recent K known to the host (sizes the MFMA column tiles)
};
void launch_assign_fp32(const Ws& ws, const AssignArgs& a, hipStream_t s);
void launch_assign_fp64(const Ws& ws, const AssignArgs& a, hipStream_t s);
struct SubArgs;
// (sub: the sweep's sub-cluster pass fused into the cluster draw, or null)
void launch_assign_bf16(const Ws& ws, const AssignArgs& a, const SubArgs* sub, hipStream_t s);
hipError_t configure_assign_bf16();
void launch_refine(const Ws& ws, const AssignArgs& a, hipStream_t s);
// FP64 scores of listed cells against the last redraw's parameters: K cluster
// columns, then the two sub-clusters of the cell's cluster c[i] (row stride K + 2)
void launch_dump_scores(const Ws& ws, const int32_t* c, const int32_t* cells, int32_t m, double* out, hipStream_t s);

// splitmerge.hip
void launch_lgamma_beta(const Ws& ws, hipStream_t s);   // lgbeta = lgamma(beta), wherever beta changes
// (k_guess below: a recent K, which sizes the grids; any K is covered)
void launch_split_ratios(const Ws& ws, const int32_t* c, const uint8_t* cs, int k_guess, hipStream_t s);
void launch_random_split(const Ws& ws, const int32_t* c, uint8_t* cs, uint32_t step, bool ready, int k_guess,
                         hipStream_t s);
void launch_merge_ratios(const Ws& ws, int k_guess, hipStream_t s);
void launch_sm_decide(const Ws& ws, int merge_pass, uint32_t step, hipStream_t s);
// collapsed log joint log p(c) + sum_k logDM(s_k) (eq. 10 with Gamma(alpha), eq. 12
// integrated against eq. 28) into ws.st->log_joint
void launch_log_joint(const Ws& ws, hipStream_t s);

// dm.hip
void launch_dm_logmarginal(const int64_t* sv, int32_t J, int32_t G, const double* beta, double* out, hipStream_t s);
void launch_dm_grad(const int64_t* sv, int32_t J, int32_t G, const double* beta, const double* g, double* grad,
                    hipStream_t s);
void launch_eb_update(const Ws& ws, hipStream_t s);
void launch_fill(double* p, int64_t n, double v, hipStream_t s);

}  // namespace dpmm
