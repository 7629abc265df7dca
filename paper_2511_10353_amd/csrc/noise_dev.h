// Device white noise: Philox-4x32-10 words -> Box-Muller deviates in binary64.
//
// The paper's step 1 (Sec. 2) asks for independent unit Gaussians per cell.
// Cell c uses Philox group g = c / 4 (key = the 64-bit seed, counter =
// (g low word, g high word, stream, 0)); words (w0, w1) give cells 4g and 4g+1
// as r cos(theta) and r sin(theta), words (w2, w3) give cells 4g+2 and 4g+3.
//
// Philox-4x32 (Salmon, Moraes, Dror, Shaw, SC'11): per round, the 64-bit
// products M0*x0 and M1*x2 are split into high/low words and the state
// becomes (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0));
// the key advances by the Weyl constants after each round; 10 rounds.
//
// Box-Muller uses only correctly rounded binary64 +, -, *, /, sqrt and exact
// bit manipulation, in a fixed order with contraction disabled, so that any
// IEEE binary64 implementation of the same sequence gives the same bits:
//   u1 = (w_a + 1) 2^-32, u2 = w_b 2^-32
//   ln u1 = e LN2 + 2 t P(t^2), u1 = m 2^e, m in [sqrt(1/2), sqrt(2)),
//           t = (m-1)/(m+1), P = sum_{k<=11} t^(2k)/(2k+1) (Horner)
//   cos/sin(2 pi u2): quadrant from the top two bits, the 30-bit remainder
//           reflected about pi/4 by an exact integer subtraction, Taylor
//           series of cos (to x^16) and sin (to x^17) on [0, pi/4] (Horner
//           in x^2), coefficients (-1)^k/(2k)! and (-1)^k/(2k+1)!.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gg {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 ctr, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit product per multiplier gives both halves
        const uint64_t p0 = (uint64_t)kPhiloxM0 * ctr.x;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * ctr.z;
        ctr = {(uint32_t)(p1 >> 32) ^ ctr.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ ctr.w ^ k1, (uint32_t)p0};
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return ctr;
}

constexpr double kLn2 = 0.6931471805599453;
constexpr double kTwoPi = 6.283185307179586;
constexpr double kSqrtHalfD = 0.7071067811865476;
constexpr double kTwoM32 = 0x1p-32;
constexpr int kAtanhTerms = 11;
constexpr int kTrigTerms = 8;

constexpr double factorial_d(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f = f * (double)i;  // exact below 2^53
    return f;
}
constexpr double atanh_coeff(int k) { return 1.0 / (double)(2 * k + 1); }
constexpr double cos_coeff(int k) { return ((k & 1) ? -1.0 : 1.0) / factorial_d(2 * k); }
constexpr double sin_coeff(int k) { return ((k & 1) ? -1.0 : 1.0) / factorial_d(2 * k + 1); }

__device__ __forceinline__ double bm_log(double u) {
#pragma clang fp contract(off)
    // u is a positive normal number: split off the exponent exactly
    const uint64_t bits = (uint64_t)__double_as_longlong(u);
    int e = (int)((bits >> 52) & 0x7FF) - 1022;
    double f = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FE0000000000000ull));
    double m = f;
    if (f < kSqrtHalfD) {
        m = f * 2.0;
        e -= 1;
    }
    const double t = (m - 1.0) / (m + 1.0);
    const double s = t * t;
    double p = atanh_coeff(kAtanhTerms);
#pragma unroll
    for (int k = kAtanhTerms - 1; k >= 0; --k) p = p * s + atanh_coeff(k);
    const double a = (double)e * kLn2;
    const double b = 2.0 * (t * p);
    return a + b;
}

__device__ __forceinline__ void bm_cos_sin(uint32_t w, double& cos_t, double& sin_t) {
#pragma clang fp contract(off)
    const uint32_t q = w >> 30;
    const uint32_t rho = w & 0x3FFFFFFFu;
    const bool direct = rho < (1u << 29);
    const uint32_t n = direct ? rho : (1u << 30) - rho;
    const double x = ((double)n * kTwoM32) * kTwoPi;
    const double z = x * x;
    double pc = cos_coeff(kTrigTerms), ps = sin_coeff(kTrigTerms);
#pragma unroll
    for (int k = kTrigTerms - 1; k >= 0; --k) {
        pc = pc * z + cos_coeff(k);
        ps = ps * z + sin_coeff(k);
    }
    const double c = pc, s = x * ps;
    const double ca = direct ? c : s;
    const double sa = direct ? s : c;
    switch (q) {
        case 0: cos_t = ca; sin_t = sa; break;
        case 1: cos_t = -sa; sin_t = ca; break;
        case 2: cos_t = -ca; sin_t = -sa; break;
        default: cos_t = sa; sin_t = -ca; break;
    }
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& ga, double& gb) {
#pragma clang fp contract(off)
    const double u1 = (double)((uint64_t)wa + 1ull) * kTwoM32;
    const double r = sqrt(-2.0 * bm_log(u1));
    double c, s;
    bm_cos_sin(wb, c, s);
    ga = r * c;
    gb = r * s;
}

// Deviates of cells 4g .. 4g+3.
__device__ __forceinline__ void noise_group(uint64_t g, uint64_t seed, uint32_t stream, double out[4]) {
    const u32x4 w = philox4x32_10({(uint32_t)g, (uint32_t)(g >> 32), stream, 0u}, (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    box_muller(w.x, w.y, out[0], out[1]);
    box_muller(w.z, w.w, out[2], out[3]);
}

}  // namespace gg
