// dm.hip -- steps a6-a7: the log Dirichlet-multinomial marginal of count
// vectors (the per-cluster factor of eq. 12 with theta integrated against the
// Dirichlet normaliser of eq. 28), its gradient with respect to a per-gene
// concentration beta (digamma sums), and the empirical-Bayes fixed-point step
// for beta that the gradient's zero defines (Minka 2000).
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

constexpr int kDmThreads = 256;

// Digamma for x > 0: recurrence psi(x) = psi(x + 1) - 1/x up to x >= 12, then
// the asymptotic expansion of Abramowitz & Stegun 6.3.18 through x^-12
// (the omitted x^-14 term is below 7e-17 there).
__device__ inline double psi(double x)
{
    double acc = 0.0;
    while (x < 12.0) {
        acc -= 1.0 / x;
        x += 1.0;
    }
    const double y = 1.0 / (x * x);
    const double series =
        y * (1.0 / 12.0 - y * (1.0 / 120.0 - y * (1.0 / 252.0 - y * (1.0 / 240.0 - y * (1.0 / 132.0 - y * (691.0 / 32760.0))))));
    return acc + log(x) - 0.5 / x - series;
}

__device__ inline double reduce_sum(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < kDmThreads / 64; ++q) s += red[q];
    __syncthreads();
    return s;
}

__device__ inline long long reduce_sum_ll(long long v, long long* red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    long long s = 0;
    for (int q = 0; q < kDmThreads / 64; ++q) s += red[q];
    __syncthreads();
    return s;
}

// out[j] = lgamma(B) - lgamma(B + S_j) + sum_u [lgamma(beta_u + s_ju) - lgamma(beta_u)]
__global__ void __launch_bounds__(kDmThreads) k_dm_logmarginal(const int64_t* __restrict__ sv, int32_t J, int32_t G,
                                                               const double* __restrict__ beta, double* __restrict__ out)
{
    __shared__ double red[kDmThreads / 64], red2[kDmThreads / 64], red3[kDmThreads / 64];
    __shared__ long long redl[kDmThreads / 64];
    for (int j = blockIdx.x; j < J; j += gridDim.x) {
        const int64_t* s = sv + (int64_t)j * G;
        double acc = 0.0, comp = 0.0, B = 0.0;
        long long S = 0;
        for (int u = threadIdx.x; u < G; u += kDmThreads) {
            B += beta[u];
            const long long v = s[u];
            if (!v) continue;
            S += v;
            const double term = lgamma(beta[u] + (double)v) - lgamma(beta[u]);
            const double tt = acc + term;
            comp += fabs(acc) >= fabs(term) ? (acc - tt) + term : (term - tt) + acc;
            acc = tt;
        }
        const double sum_terms = reduce_sum(acc, red) + reduce_sum(comp, red2);
        const double Bt = reduce_sum(B, red3);
        const long long St = reduce_sum_ll(S, redl);
        if (threadIdx.x == 0) out[j] = (lgamma(Bt) - lgamma(Bt + (double)St)) + sum_terms;
    }
}

// grad[u] = sum_j g_j [psi(B) - psi(B + S_j)] + sum_j g_j [psi(beta_u + s_ju) - psi(beta_u)]
// Every workgroup recomputes B and the J totals S_j (J x G reads, small) so
// that the call needs no scratch memory.
__global__ void __launch_bounds__(kDmThreads) k_dm_grad(const int64_t* __restrict__ sv, int32_t J, int32_t G,
                                                        const double* __restrict__ beta, const double* __restrict__ g,
                                                        double* __restrict__ grad)
{
    __shared__ double red[kDmThreads / 64];
    __shared__ long long redl[kDmThreads / 64];
    double B = 0.0;
    for (int u = threadIdx.x; u < G; u += kDmThreads) B += beta[u];
    B = reduce_sum(B, red);
    const double psiB = psi(B);
    double common = 0.0;
    for (int j = 0; j < J; ++j) {
        long long S = 0;
        for (int u = threadIdx.x; u < G; u += kDmThreads) S += sv[(int64_t)j * G + u];
        S = reduce_sum_ll(S, redl);
        common += g[j] * (psiB - psi(B + (double)S));
    }
    for (int u = blockIdx.x * kDmThreads + threadIdx.x; u < G; u += gridDim.x * kDmThreads) {
        const double bu = beta[u];
        const double pb = psi(bu);
        double acc = common;
        for (int j = 0; j < J; ++j) {
            const long long v = sv[(int64_t)j * G + u];
            if (v) acc += g[j] * (psi(bu + (double)v) - pb);
        }
        grad[u] = acc;
    }
}

void launch_dm_logmarginal(const int64_t* sv, int32_t J, int32_t G, const double* beta, double* out, hipStream_t s)
{
    const int blocks = J < 4096 ? J : 4096;
    hipLaunchKernelGGL(k_dm_logmarginal, dim3(blocks > 0 ? blocks : 1), dim3(kDmThreads), 0, s, sv, J, G, beta, out);
}

void launch_dm_grad(const int64_t* sv, int32_t J, int32_t G, const double* beta, const double* g, double* grad,
                    hipStream_t s)
{
    const int blocks = (G + kDmThreads - 1) / kDmThreads;
    hipLaunchKernelGGL(k_dm_grad, dim3(blocks > 0 ? blocks : 1), dim3(kDmThreads), 0, s, sv, J, G, beta, g, grad);
}

// ---------------------------------------------------------------------------
// Empirical-Bayes step over the K current clusters (statistics
// s_k = s_{k,0} + s_{k,1}):
//   beta_u <- beta_u * sum_k [psi(s_ku + beta_u) - psi(beta_u)] / sum_k [psi(S_k + B) - psi(B)],
// clamped to [1e-6, 1e6].  Phase 1 (one workgroup per cluster) writes the
// denominator terms; phase 2 (one thread per gene) updates beta in place,
// after every workgroup of phase 1 has read the old B.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kDmThreads) k_eb_denominator(Ws ws)
{
    __shared__ double red[kDmThreads / 64];
    __shared__ long long redl[kDmThreads / 64];
    const int K = ws.st->K;
    const int G = ws.G;
    for (int k = blockIdx.x; k < K; k += gridDim.x) {
        double B = 0.0;
        long long S = 0;
        for (int u = threadIdx.x; u < G; u += kDmThreads) {
            B += ws.beta[u];
            S += (long long)(ws.ssub[(int64_t)(2 * k) * G + u] + ws.ssub[(int64_t)(2 * k + 1) * G + u]);
        }
        B = reduce_sum(B, red);
        S = reduce_sum_ll(S, redl);
        if (threadIdx.x == 0) ws.eb_tmp[k] = psi((double)S + B) - psi(B);
    }
}

__global__ void __launch_bounds__(kDmThreads) k_eb_update(Ws ws)
{
    const int K = ws.st->K;
    const int G = ws.G;
    double den = 0.0;
    for (int k = 0; k < K; ++k) den += ws.eb_tmp[k];
    for (int u = blockIdx.x * kDmThreads + threadIdx.x; u < G; u += gridDim.x * kDmThreads) {
        const double b = ws.beta[u];
        const double pb = psi(b);
        double num = 0.0;
        for (int k = 0; k < K; ++k) {
            const long long v = (long long)(ws.ssub[(int64_t)(2 * k) * G + u] + ws.ssub[(int64_t)(2 * k + 1) * G + u]);
            if (v) num += psi((double)v + b) - pb;
        }
        const double x = den > 0.0 ? b * num / den : b;
        ws.beta[u] = fmin(1e6, fmax(1e-6, x));
    }
}

void launch_eb_update(const Ws& ws, hipStream_t s)
{
    const int kb = ws.k_max < 1024 ? ws.k_max : 1024;
    hipLaunchKernelGGL(k_eb_denominator, dim3(kb), dim3(kDmThreads), 0, s, ws);
    const int blocks = (ws.G + kDmThreads - 1) / kDmThreads;
    hipLaunchKernelGGL(k_eb_update, dim3(blocks), dim3(kDmThreads), 0, s, ws);
    launch_lgamma_beta(ws, s);
}

__global__ void k_fill(double* p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void launch_fill(double* p, int64_t n, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
}

}  // namespace dpmm
