// redraw.hip -- step a1: draw pi ~ Dir(n_1..n_K, alpha), theta_k ~ Dir(beta + s_k)
// and thetabar_{k,r} ~ Dir(beta + s_{k,r}) (Section 2.1 eq. 4, first two
// lines; Section 2.3 eq. 19 with lambdabar = lambda), in FP64 and in log space.
// One workgroup per parameter row; the row is also written in the layouts the
// assignment kernels read (FP32 gene-major tables, split-BF16 hi/lo).
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

// Log of a Gamma(a, 1) variate: Marsaglia & Tsang (2000) with Box-Muller
// normals; a < 1 uses Gamma(a) = Gamma(a + 1) U^(1/a), added in log space.
// Attempt j reads counter calls 2j (normal) and 2j + 1 (acceptance uniform,
// boost uniform).  The log-acceptance 0.5 z^2 + d - d v + d log v is written
// through t = c z, v = (1 + t)^3, so large shapes do not cancel.
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
    *capped = 1;
    return log(d);
}

constexpr int kRedrawThreads = 256;

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

__global__ void __launch_bounds__(kRedrawThreads) k_redraw(Ws ws, uint32_t step, int write_split)
{
    __shared__ double red[kRedrawThreads / 64];
    const int K = ws.st->K;
    const int row = blockIdx.x;
    const int G = ws.G;
    const int t = threadIdx.x;
    int capped = 0;

    if (row == 3 * ws.k_max) {
        if (t == 0) ws.st->counters[kCntEvals] += (unsigned long long)ws.N * (unsigned long long)(K + 2);
        // mixing proportions: Gamma(n_k) for the K clusters and Gamma(alpha)
        double* lp = ws.logpi;
        double m = -INFINITY;
        double lga = -INFINITY;
        for (int k = t; k <= K; k += kRedrawThreads) {
            double v;
            if (k < K) {
                const double n = (double)(ws.nsub[2 * k] + ws.nsub[2 * k + 1]);
                v = log_gamma_draw(n, ws.seed, (uint32_t)k, 0u, step, kPi, &capped);
                lp[k] = v;
            } else {
                v = log_gamma_draw(ws.alpha, ws.seed, kAlphaElement, 0u, step, kPi, &capped);
                lga = v;
            }
            m = fmax(m, v);
        }
        m = block_max(m, red);
        double s = 0.0;
        for (int k = t; k < K; k += kRedrawThreads) s += exp(lp[k] - m);
        if (K % kRedrawThreads == t) s += exp(lga - m);
        const double lse = m + log(block_sum(s, red));
        for (int k = t; k < K; k += kRedrawThreads) lp[k] -= lse;
        if (capped) atomicAdd(&ws.st->counters[kCntGammaCaps], 1ull);
        return;
    }

    int k, r = -1;
    uint32_t philox_row;
    double* out;
    if (row < ws.k_max) {
        k = row;
        if (k >= K) return;
        philox_row = (uint32_t)k;
        out = ws.lt64 + (int64_t)k * G;
    } else {
        const int q = row - ws.k_max;     // q = 2k + r
        if (q >= 2 * K) return;
        k = q >> 1;
        r = q & 1;
        philox_row = kSubRowBase + (uint32_t)q;
        out = ws.lt64 + (int64_t)row * G;
    }
    const unsigned long long* s0 = ws.ssub + (int64_t)(2 * k) * G;
    const unsigned long long* s1 = s0 + G;

    double m = -INFINITY;
    for (int u = t; u < G; u += kRedrawThreads) {
        const unsigned long long cnt = r < 0 ? s0[u] + s1[u] : (r == 0 ? s0[u] : s1[u]);
        const double v = log_gamma_draw(ws.beta[u] + (double)cnt, ws.seed, (uint32_t)u, philox_row, step, kGamma,
                                        &capped);
        out[u] = v;
        m = fmax(m, v);
    }
    m = block_max(m, red);
    double s = 0.0;
    for (int u = t; u < G; u += kRedrawThreads) s += exp(out[u] - m);
    const double lse = m + log(block_sum(s, red));
    float* ls = reinterpret_cast<float*>(ws.ls32);
    for (int u = t; u < G; u += kRedrawThreads) {
        const double v = out[u] - lse;
        out[u] = v;
        if (r < 0) {
            ws.lc32[(int64_t)u * ws.kpad + k] = (float)v;
            if (write_split) {
                // split-BF16: hi = bf16(v), lo = bf16(v - hi), cluster-major
                // [k][Gpad] as the MFMA kernel stages them
                const float f = (float)v;
                const uint16_t hi = bf16_bits(f);
                const uint16_t lo = bf16_bits((float)(v - (double)bf16_value(hi)));
                ws.lhi[(int64_t)k * ws.Gpad + u] = hi;
                ws.llo[(int64_t)k * ws.Gpad + u] = lo;
            }
        } else {
            ls[((int64_t)u * ws.k_max + k) * 2 + r] = (float)v;
        }
    }
    if (capped) atomicAdd(&ws.st->counters[kCntGammaCaps], 1ull);
}

void launch_redraw(const Ws& ws, uint32_t step, int write_split, hipStream_t s)
{
    hipLaunchKernelGGL(k_redraw, dim3((unsigned)(3 * ws.k_max + 1)), dim3(kRedrawThreads), 0, s, ws, step,
                       write_split);
}

}  // namespace dpmm
