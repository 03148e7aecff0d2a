// redraw.hip -- step a1: draw pi ~ Dir(n_1..n_K, alpha), theta_k ~ Dir(beta + s_k)
// and thetabar_{k,r} ~ Dir(beta + s_{k,r}) (Section 2.1 eq. 4, first two
// lines; Section 2.3 eq. 19 with lambdabar = lambda), in FP64 and in log space.
// Two passes over (row, tile of genes) workgroups: the Gamma variates with
// per-tile partial sums, then the normalisation; each row is also written in
// the layouts the assignment kernels read (FP32 gene-major tables, split-BF16
// hi/lo).
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

// Log of a Gamma(a, 1) variate: Marsaglia & Tsang (2000) with Box-Muller
// normals; a < 1 uses Gamma(a) = Gamma(a + 1) U^(1/a), added in log space.
// Attempt j reads counter calls 2j (normal) and 2j + 1 (acceptance uniform,
// boost uniform).  The log-acceptance 0.5 z^2 + d - d v + d log v is written
// through t = c z, v = (1 + t)^3, so large shapes do not cancel.  A draw
// that exhausts kGammaTries attempts adds one to *capped.
__device__ double log_gamma_draw(double a, uint64_t seed, uint32_t element, uint32_t row, uint32_t step,
                                 uint32_t stream, int* capped)
{
    const bool boost = a < 1.0;
    const double d = (boost ? a + 1.0 : a) - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    for (int j = 0; j < kGammaTries; ++j) {
        const Words nw = philox(seed, element, row, step, stream, 2u * (uint32_t)j);
        const double r1 = unit52(nw.w[0], nw.w[1]);
        const double r2 = unit52(nw.w[2], nw.w[3]);
        const double z = sqrt(-2.0 * log(r1)) * cos(6.283185307179586 * r2);
        const double t = c * z;
        if (t <= -1.0) continue;
        const Words aw = philox(seed, element, row, step, stream, 2u * (uint32_t)j + 1u);
        const double lu = log(unit52(aw.w[0], aw.w[1]));
        const double l1t = log1p(t);
        const double bound = 0.5 * z * z + d * (3.0 * l1t - t * (3.0 + t * (3.0 + t)));
        if (lu < bound) {
            double out = log(d) + 3.0 * l1t;
            if (boost) out += log(unit52(aw.w[2], aw.w[3])) / a;
            return out;
        }
    }
    *capped += 1;
    return log(d);
}

constexpr int kRedrawThreads = 256;
static_assert(kRedrawThreads == kRedrawGenes, "one gene per thread in the redraw passes");

__device__ inline double block_max(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double m = red[0];
    for (int q = 1; q < kRedrawThreads / 64; ++q) m = fmax(m, red[q]);
    __syncthreads();
    return m;
}

__device__ inline double block_sum(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int q = 1; q < kRedrawThreads / 64; ++q) s += red[q];
    __syncthreads();
    return s;
}

// bf16 bit pattern of a float, round to nearest even (finite inputs)
__device__ inline uint16_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// The row a workgroup redraws: cluster k (r < 0) or sub-cluster (k, r);
// false when the row is past the current K.
struct RedrawRow {
    int k, r;
    uint32_t philox_row;
    double* out;
};

__device__ inline bool redraw_row(const Ws& ws, int row, int K, RedrawRow& rr)
{
    if (row < ws.k_max) {
        if (row >= K) return false;
        rr.k = row;
        rr.r = -1;
        rr.philox_row = (uint32_t)row;
    } else {
        const int q = row - ws.k_max;     // q = 2k + r
        if (q >= 2 * K) return false;
        rr.k = q >> 1;
        rr.r = q & 1;
        rr.philox_row = kSubRowBase + (uint32_t)q;
    }
    rr.out = ws.lt64 + (int64_t)row * ws.G;
    return true;
}

// The rows a sweep redraws, as virtual rows v: the K cluster rows (v < K),
// then the 2K sub-cluster rows (row k_max + v - K).  The grid is sized from
// the host's recent K and loops when K has grown past it; its last column
// draws log pi.
__device__ inline int redraw_vrow(const Ws& ws, int v, int K)
{
    return v < K ? v : ws.k_max + (v - K);
}

// Pass 1, one workgroup per (virtual row, tile of kRedrawGenes genes): the log
// Gamma variates of the tile, and the tile's (max, sum exp(v - max)).  Log pi
// is drawn and normalised by tile 0 of the grid's last column.
__global__ void __launch_bounds__(kRedrawThreads) k_redraw_draw(Ws ws, uint32_t step)
{
    __shared__ double red[kRedrawThreads / 64];
    const int K = ws.st->K;
    const int tile = blockIdx.y;
    const int G = ws.G;
    const int t = threadIdx.x;
    const int nrow = (int)gridDim.x - 1;        // columns of the gene rows
    int capped = 0;

    if ((int)blockIdx.x == nrow) {
        if (tile != 0) return;
        if (t == 0) atomicAdd(&ws.st->counters[kCntEvals], (unsigned long long)ws.N * (unsigned long long)(K + 2));
        double* lp = ws.logpi;
        // with a new cluster in the sweep (eq. 4 over K + 1) the alpha
        // component is its weight
        const int Kc = ws.st->has_new ? K - 1 : K;     // clusters with cells
        double m = -INFINITY;
        double lga = -INFINITY;
        for (int k = t; k <= Kc; k += kRedrawThreads) {
            double v;
            if (k < Kc) {
                const double n = (double)(ws.nsub[2 * k] + ws.nsub[2 * k + 1]);
                v = log_gamma_draw(n, ws.seed, (uint32_t)k, 0u, step, kPi, &capped);
                lp[k] = v;
            } else {
                v = log_gamma_draw(ws.alpha, ws.seed, kAlphaElement, 0u, step, kPi, &capped);
                lga = v;
                if (Kc < K) lp[Kc] = v;
            }
            m = fmax(m, v);
        }
        m = block_max(m, red);
        double s = 0.0;
        for (int k = t; k < Kc; k += kRedrawThreads) s += exp(lp[k] - m);
        if (Kc % kRedrawThreads == t) s += exp(lga - m);
        const double lse = m + log(block_sum(s, red));
        __syncthreads();
        for (int k = t; k < K; k += kRedrawThreads) lp[k] -= lse;
        if (capped) atomicAdd(&ws.st->counters[kCntGammaCaps], (unsigned long long)capped);
        return;
    }

    const int u = tile * kRedrawGenes + t;
#pragma unroll 1
    for (int vr = blockIdx.x; vr < 3 * K; vr += nrow) {
        const int row = redraw_vrow(ws, vr, K);
        RedrawRow rr;
        redraw_row(ws, row, K, rr);
        const unsigned long long* s0 = ws.ssub + (int64_t)(2 * rr.k) * G;
        const unsigned long long* s1 = s0 + G;
        double v = -INFINITY;
        if (u < G) {
            const unsigned long long cnt = rr.r < 0 ? s0[u] + s1[u] : (rr.r == 0 ? s0[u] : s1[u]);
            v = log_gamma_draw(ws.beta[u] + (double)cnt, ws.seed, (uint32_t)u, rr.philox_row, step, kGamma, &capped);
            rr.out[u] = v;
        }
        const double m = block_max(v, red);
        const double s = block_sum(u < G ? exp(v - m) : 0.0, red);
        if (t == 0) ws.rd_part[(int64_t)row * redraw_tiles(G) + tile] = make_double2(m, s);
    }
    if (capped) atomicAdd(&ws.st->counters[kCntGammaCaps], (unsigned long long)capped);
}

// Pass 2, same grid: the row's log normaliser from its tiles' partials
// (combined in tile order), then the tile's log theta in FP64 and in the
// layouts the assignment kernels read.
//
// The whole grid also prepares the sweep's counts (saving a launch): the
// counts at the start of the sweep, which feed eq. 8, move to nsub_prev, and
// the new counts, statistics and sort counters start from zero.  Pass 1 has
// read them; nothing else reads them before the sub-cluster pass rebuilds them.
// With zero_rs the coin-half statistics (rssub / rnsub) start from zero too:
// the sub-cluster pass of this sweep gathers them for the random split that
// follows it.
__global__ void __launch_bounds__(kRedrawThreads) k_redraw_norm(Ws ws, int write_split, int zero_rs)
{
    const int K = ws.st->K;
    // the re-score queue of the sweep that follows starts empty
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) ws.st->n_refine = ws.st->n_mov = 0;
    {
        const int64_t nt = (int64_t)gridDim.x * gridDim.y * blockDim.x;
        const int64_t t0 = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
        for (int64_t q = t0; q < 2 * (int64_t)ws.k_max; q += nt) {
            ws.nsub_prev[q] = ws.nsub[q];
            ws.nsub[q] = 0;
        }
        for (int64_t q = t0; q < ws.k_max; q += nt) ws.grp_cnt[q] = 0;
        ulonglong2* sv = reinterpret_cast<ulonglong2*>(ws.ssub);      // 2 k_max G is even
        for (int64_t q = t0; q < (int64_t)ws.k_max * ws.G; q += nt) sv[q] = make_ulonglong2(0ull, 0ull);
        if (zero_rs) {
            ulonglong2* rv = reinterpret_cast<ulonglong2*>(ws.rssub);
            for (int64_t q = t0; q < (int64_t)ws.k_max * ws.G; q += nt) rv[q] = make_ulonglong2(0ull, 0ull);
            for (int64_t q = t0; q < 2 * (int64_t)ws.k_max; q += nt) ws.rnsub[q] = 0;
        }
    }
    const int tile = blockIdx.y;
    const int G = ws.G;
    const int t = threadIdx.x;
    const int nt = redraw_tiles(G);
    const int u = tile * kRedrawGenes + t;
    // the virtual rows of pass 1, by the same columns (the last one, log pi's,
    // has nothing to do here)
    const int nrow = (int)gridDim.x - 1;
    if ((int)blockIdx.x == nrow) return;
    for (int vr = blockIdx.x; vr < 3 * K; vr += nrow) {
        const int row = redraw_vrow(ws, vr, K);
        RedrawRow rr;
        redraw_row(ws, row, K, rr);
        const double2* part = ws.rd_part + (int64_t)row * nt;
        double m = -INFINITY;
#pragma unroll 8
        for (int q = 0; q < nt; ++q) m = fmax(m, part[q].x);
        double s = 0.0;
#pragma unroll 8
        for (int q = 0; q < nt; ++q) s += part[q].y * exp(part[q].x - m);
        const double lse = m + log(s);
        if (u >= G) continue;
        const double v = rr.out[u] - lse;
        rr.out[u] = v;
        const int k = rr.k;
        if (rr.r < 0) {
            ws.lc32[(int64_t)u * ws.kpad + k] = (float)v;
            if (write_split) {
                const float f = (float)v;
                const uint16_t hi = bf16_bits(f);
                const uint16_t lo = bf16_bits((float)(v - (double)bf16_value(hi)));
                ws.lhi[(int64_t)k * ws.Gpad + u] = hi;
                ws.llo[(int64_t)k * ws.Gpad + u] = lo;
            }
        } else {
            reinterpret_cast<float*>(ws.ls32)[((int64_t)u * ws.k_max + k) * 2 + rr.r] = (float)v;
        }
    }
}

void launch_redraw(const Ws& ws, uint32_t step, int write_split, int zero_rs, int k_guess, hipStream_t s)
{
    // rows for a sweep over k_guess clusters (the kernels loop past it)
    const int kg = k_guess > 0 && k_guess < ws.k_max ? k_guess : ws.k_max;
    const dim3 grid((unsigned)(3 * kg + 1), (unsigned)redraw_tiles(ws.G));
    hipLaunchKernelGGL(k_redraw_draw, grid, dim3(kRedrawThreads), 0, s, ws, step);
    hipLaunchKernelGGL(k_redraw_norm, grid, dim3(kRedrawThreads), 0, s, ws, write_split,
                       zero_rs && ws.rssub != nullptr ? 1 : 0);
}

}  // namespace dpmm
