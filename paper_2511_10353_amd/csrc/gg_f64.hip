// Double-precision instantiation of the kernels and launchers, and the FP64
// sigma_8 integral.
#include "ops_impl.h"

namespace gg {
template struct Ops<double>;

// out[0] = S (the sigma^2(8 Mpc/h) of the spectrum with A = 1)
__global__ __launch_bounds__(kSigmaThreads) void k_sigma_integral(double lnk_min, double lnk_max, double gamma,
                                                                   double n_s, double radius, double* out) {
    __shared__ double part[kSigmaThreads];
    const double h = (lnk_max - lnk_min) / kSimpsonIntervals;
    double acc = 0.0;
    for (int i = threadIdx.x; i <= kSimpsonIntervals; i += kSigmaThreads) {
        const double lnk = (i == kSimpsonIntervals) ? lnk_max : lnk_min + (double)i * h;
        const double k = exp(lnk);
        const double t = bbks(k, gamma);
        const double w = tophat(k * radius);
        const double f = k * k * k * pow(k, n_s) * t * t * w * w;
        const double wt = (i == 0 || i == kSimpsonIntervals) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
        acc += wt * f;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kSigmaThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0] * h / 3.0 / (2.0 * kPi * kPi);
}


constexpr int kDotThreads = 1024;

// out = scale * sum of part[0..count), one work-group, fixed order (eight
// independent partial sums per thread keep eight loads in flight)
__global__ __launch_bounds__(kDotThreads) void k_dot_final(const double* __restrict__ part, uint32_t count,
                                                           double scale, double* __restrict__ out) {
    __shared__ double red[kDotThreads];
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    uint32_t i = threadIdx.x;
    for (; i + 7 * kDotThreads < count; i += 8 * kDotThreads) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += part[i + u * kDotThreads];
    }
    for (int u = 0; i < count; i += kDotThreads, ++u) acc[u] += part[i];
    red[threadIdx.x] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] * scale;
}

void refine_sizes(int variant, int& nl, int& nh) {
    switch (variant) {
        case REFINE_HR: nl = RefineBasis<REFINE_HR>::NL; nh = RefineBasis<REFINE_HR>::NH; break;
        case REFINE_3: nl = RefineBasis<REFINE_3>::NL; nh = RefineBasis<REFINE_3>::NH; break;
        case REFINE_4: nl = RefineBasis<REFINE_4>::NL; nh = RefineBasis<REFINE_4>::NH; break;
        case REFINE_LINEAR: nl = RefineBasis<REFINE_LINEAR>::NL; nh = RefineBasis<REFINE_LINEAR>::NH; break;
        case REFINE_SINE: nl = RefineBasis<REFINE_SINE>::NL; nh = RefineBasis<REFINE_SINE>::NH; break;
        default: nl = nh = 0;
    }
}

hipError_t launch_dot_final(const double* part, uint32_t count, double scale, double* out, hipStream_t s) {
    k_dot_final<<<1, kDotThreads, 0, s>>>(part, count, scale, out);
    return hipGetLastError();
}

hipError_t launch_sigma_integral(double lnk_min, double lnk_max, double gamma, double n_s, double radius,
                                 double* out, hipStream_t s) {
    k_sigma_integral<<<1, kSigmaThreads, 0, s>>>(lnk_min, lnk_max, gamma, n_s, radius, out);
    return hipGetLastError();
}
}  // namespace gg
