// FP64 device kernels for the spectrum normalisation and the filter table.
//
// Spectrum (the paper takes P(k) as a table, Sec. 2.1; the workloads use an
// analytic stand-in): P(k, z) = D(z)^2 A k^n_s T(k)^2 with the BBKS transfer
// function (Bardeen, Bond, Kaiser & Szalay 1986, eq. G3), q = k / Gamma:
//   T = ln(1 + 2.34 q)/(2.34 q) [1 + 3.89 q + (16.1 q)^2 + (5.46 q)^3 + (6.71 q)^4]^(-1/4).
// sigma_8 normalisation (Sec. 2.1 footnote): A = sigma_8^2 / S with
//   S = (1/2 pi^2) int k^3 k^n_s T^2 W(8k)^2 d ln k,  W(x) = 3 (sin x - x cos x)/x^3,
// composite Simpson over ln k in [ln 1e-5, ln 1e3] with 2^16 intervals,
// summed by one work-group in a fixed order (deterministic).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gg {

constexpr int kSimpsonIntervals = 1 << 16;
constexpr int kSigmaThreads = 1024;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double bbks(double k, double gamma) {
    const double q = k / gamma;
    const double aq = 2.34 * q;
    const double lead = aq < 1e-8 ? 1.0 - 0.5 * aq : log1p(aq) / aq;
    const double p2 = 16.1 * q, p3 = 5.46 * q, p4 = 6.71 * q;
    const double poly = 1.0 + 3.89 * q + p2 * p2 + p3 * p3 * p3 + (p4 * p4) * (p4 * p4);
    return lead * pow(poly, -0.25);
}

__device__ __forceinline__ double tophat(double x) {
    if (x < 1e-2) return 1.0 - x * x / 10.0 + x * x * x * x / 280.0;
    return 3.0 * (sin(x) - x * cos(x)) / (x * x * x);
}

// tau[n2] = (L / 2 pi) sqrt(P(k) N^3 / L^3) / (n2 N^3), k = (2 pi / L) sqrt(n2);
// tau[0] = 0.  Evaluated in binary64 and rounded once to T.
template <typename T>
__global__ void k_tau(T* __restrict__ tau, int64_t ntau, int n, double box, double amp_growth2, double gamma,
                      double n_s) {
    const double n3 = (double)n * (double)n * (double)n;
    const double kf = 2.0 * kPi / box;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntau; i += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (i > 0) {
            const double n2 = (double)i;
            const double k = kf * sqrt(n2);
            const double t = bbks(k, gamma);
            const double p = amp_growth2 * pow(k, n_s) * t * t;
            v = (box / (2.0 * kPi)) * sqrt(p * n3 / (box * box * box)) / (n2 * n3);
        }
        tau[i] = (T)v;
    }
}

}  // namespace gg
