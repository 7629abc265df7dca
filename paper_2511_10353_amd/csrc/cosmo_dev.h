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

// tau(x) = (L / 2 pi) sqrt(P(k) N^3 / L^3) / (x N^3), k = (2 pi / L) sqrt(x),
// for real x > 0 (x = n^2 on the lattice).
__device__ __forceinline__ double tau_value(double x, double n3, double box, double amp_growth2, double gamma,
                                            double n_s) {
    const double k = (2.0 * kPi / box) * sqrt(x);
    const double t = bbks(k, gamma);
    const double p = amp_growth2 * pow(k, n_s) * t * t;
    return (box / (2.0 * kPi)) * sqrt(p * n3 / (box * box * box)) / (x * n3);
}

// tau[n2] = tau_value(n2), tau[0] = 0.  Evaluated in binary64 and rounded
// once to T.
template <typename T>
__global__ void k_tau(T* __restrict__ tau, int64_t ntau, int n, double box, double amp_growth2, double gamma,
                      double n_s) {
    const double n3 = (double)n * (double)n * (double)n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntau; i += (int64_t)gridDim.x * blockDim.x)
        tau[i] = i > 0 ? (T)tau_value((double)i, n3, box, amp_growth2, gamma, n_s) : (T)0;
}

// Piecewise-cubic form of tau for the single-precision fused passes, small
// enough (15 KB) to sit in LDS next to a transform tile.  Integer n2 < 2^20
// maps to segment seg(n2) = 64 sh + (n2 >> sh), sh = max(floor(log2 n2) - 6, 0),
// and t = (n2 mod 2^sh) / 2^sh in [0, 1): segments below 128 hold single
// integers (exact values), above that each octave is cut into 64 segments of
// width 2^sh.  Segment coefficients (c0, c1, c2, c3) interpolate tau(x) at
// t = 0, 1/3, 2/3, 1 (Newton forward differences in binary64, rounded to
// float); tau ~ x^-a with a < 2 varies by < 4% over a segment, so the cubic's
// relative error is below 1e-8, under float rounding.
constexpr int kTauSeg = 64 * 15;  // n2 < 2^20 covers N <= 1024

template <typename T>  // T: the plan's type (instantiated per translation unit)
__global__ void k_tauseg(float4* __restrict__ seg, int n, double box, double amp_growth2, double gamma,
                         double n_s) {
    const double n3 = (double)n * (double)n * (double)n;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < kTauSeg; s += gridDim.x * blockDim.x) {
        float4 c = {0.f, 0.f, 0.f, 0.f};
        if (s < 128) {
            if (s > 0) c.x = (float)tau_value((double)s, n3, box, amp_growth2, gamma, n_s);
        } else {
            const int sh = (s >> 6) - 1;
            const double base = (double)((s & 63) + 64) * (double)(1 << sh);
            const double w = (double)(1 << sh);
            double f[4];
            for (int i = 0; i < 4; ++i) f[i] = tau_value(base + w * i / 3.0, n3, box, amp_growth2, gamma, n_s);
            const double d1 = f[1] - f[0];
            const double d2 = f[2] - 2.0 * f[1] + f[0];
            const double d3 = f[3] - 3.0 * f[2] + 3.0 * f[1] - f[0];
            c.x = (float)f[0];
            c.y = (float)(3.0 * d1 - 1.5 * d2 + d3);
            c.z = (float)(4.5 * d2 - 4.5 * d3);
            c.w = (float)(4.5 * d3);
        }
        seg[s] = c;
    }
}

// Piecewise degree-7 form of tau for the double-precision fused passes, 32 KB
// in LDS next to a 128 KB transform tile.  Integer n2 < 2^20 maps to segment
// seg(n2) = 32 sh + (n2 >> sh), sh = max(floor(log2 n2) - 5, 0), and
// t = (n2 mod 2^sh) / 2^sh in [0, 1): segments below 64 hold single integers
// (exact values), above that each octave is cut into 32 segments of width
// 2^sh.  Segment s stores the monomial coefficients c0..c7 (in t) of the
// polynomial interpolating tau at the eight Chebyshev points of [0, 1]
// (Newton divided differences in binary64, expanded); the relative error is
// below 2e-15 for every n2 of lattices from 16^3 to 1024^3 and boxes from 60
// to 5000 Mpc/h, against the 1e-12 bar of the double path.
constexpr int kTauSeg64 = 32 * 16;  // n2 < 2^20 covers N <= 1024
constexpr int kTauDeg64 = 7;

template <typename T>  // T: the plan's type (instantiated per translation unit)
__global__ void k_tauseg64(double* __restrict__ coef, int n, double box, double amp_growth2, double gamma,
                           double n_s) {
    constexpr int K = kTauDeg64 + 1;
    const double n3 = (double)n * (double)n * (double)n;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < kTauSeg64; s += gridDim.x * blockDim.x) {
        double c[K];
        for (int k = 0; k < K; ++k) c[k] = 0.0;
        if (s < 64) {
            if (s > 0) c[0] = tau_value((double)s, n3, box, amp_growth2, gamma, n_s);
        } else {
            const int sh = (s >> 5) - 1;
            const double w = (double)(1 << sh);
            const double base = (double)((s & 31) + 32) * w;
            double tn[K], f[K];
            for (int i = 0; i < K; ++i) {
                tn[i] = 0.5 - 0.5 * cos(kPi * (i + 0.5) / K);
                f[i] = tau_value(base + w * tn[i], n3, box, amp_growth2, gamma, n_s);
            }
            for (int j = 1; j < K; ++j)  // divided differences f[t0..ti] in place
                for (int i = K - 1; i >= j; --i) f[i] = (f[i] - f[i - 1]) / (tn[i] - tn[i - j]);
            // p(t) = f0 + (t - t0)(f1 + (t - t1)(f2 + ...)), expanded from the inside out
            c[0] = f[K - 1];
            int deg = 0;
            for (int i = K - 2; i >= 0; --i) {
                // c <- c * (t - tn[i]) + f[i]
                c[deg + 1] = c[deg];
                for (int k = deg; k >= 1; --k) c[k] = c[k - 1] - tn[i] * c[k];
                c[0] = f[i] - tn[i] * c[0];
                ++deg;
            }
        }
        for (int k = 0; k < K; ++k) coef[(size_t)s * K + k] = c[k];
    }
}

}  // namespace gg
