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
// Box-Muller uses only correctly rounded +, -, *, /, sqrt and exact bit
// manipulation, in a fixed order with contraction disabled, so that any IEEE
// implementation of the same sequence gives the same bits.  The double path
// evaluates it in binary64:
//   u1 = (w_a + 1) 2^-32, u2 = w_b 2^-32
//   ln u1 = e LN2 + 2 t P(t^2), u1 = m 2^e, m in [sqrt(1/2), sqrt(2)),
//           t = (m-1)/(m+1), P = sum_{k<=11} t^(2k)/(2k+1) (Horner)
//   cos/sin(2 pi u2): quadrant from the top two bits, the 30-bit remainder
//           reflected about pi/4 by an exact integer subtraction, Taylor
//           series of cos (to x^16) and sin (to x^17) on [0, pi/4] (Horner
//           in x^2), coefficients (-1)^k/(2k)! and (-1)^k/(2k+1)!.
// The float path evaluates the same structure in binary32 with series cut to
// float32 accuracy (atanh 5, cos 6, sin 5 coefficients); for u1 > sqrt(1/2)
// (w_a >= 0xB504F333) its t = (u1-1)/(u1+1) is formed from the exact integer
// d = 2^32 - 1 - w_a as -RN(d)/RN(2^33 - d), otherwise u1 = RN(w_a + 1) 2^-32;
// RN is one rounding of an integer to float32.  Constants are the float32
// roundings of the binary64 constants.
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
    const double c0 = (q & 1u) ? sa : ca;
    const double s0 = (q & 1u) ? ca : sa;
    cos_t = (q == 1u || q == 2u) ? -c0 : c0;
    sin_t = (q >= 2u) ? -s0 : s0;
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

// ---- binary32 variant --------------------------------------------------------
constexpr float kLn2F = (float)0.6931471805599453;
constexpr float kTwoPiF = (float)6.283185307179586;
constexpr float kSqrtHalfF = (float)0.7071067811865476;
constexpr float kTwoM32F = 0x1p-32f;
constexpr uint32_t kWordSplit = 0xB504F333u;  // smallest w_a with (w_a + 1) 2^-32 > sqrt(1/2)
constexpr int kAtanhTermsF = 4;
constexpr int kCosTermsF = 5;
constexpr int kSinTermsF = 4;
constexpr float atanh_coeff_f(int k) { return 1.0f / (float)(2 * k + 1); }
constexpr float cos_coeff_f(int k) { return ((k & 1) ? -1.0f : 1.0f) / (float)factorial_d(2 * k); }
constexpr float sin_coeff_f(int k) { return ((k & 1) ? -1.0f : 1.0f) / (float)factorial_d(2 * k + 1); }

__device__ __forceinline__ float bm_log_word_f(uint32_t wa) {
#pragma clang fp contract(off)
    // both reductions are formed for every lane (no divergent branch); each
    // lane divides its own numerator/denominator pair once
    const bool near_one = wa >= kWordSplit;
    const uint32_t d = 0xFFFFFFFFu - wa;
    const float dn = (float)d;  // d < 2^31: one rounding
    // RN(2^33 - d): 2^33 - d lies in (2^32, 2^33], float spacing 512 there;
    // round to nearest, ties to even, in integers
    const uint64_t x = (1ull << 33) - (uint64_t)d;
    uint32_t qd = (uint32_t)(x >> 9);
    const uint32_t rem = (uint32_t)x & 511u;
    qd += (rem > 256u || (rem == 256u && (qd & 1u))) ? 1u : 0u;
    const float dd = (float)qd * 512.0f;  // qd <= 2^24: exact
    const float u = (float)(wa + 1u) * kTwoM32F;  // used only when wa < kWordSplit
    const uint32_t bits = __float_as_uint(u);
    int ei = (int)((bits >> 23) & 0xFF) - 126;
    const float f = __uint_as_float((bits & 0x007FFFFFu) | 0x3F000000u);
    const bool low = f < kSqrtHalfF;
    const float m = low ? f * 2.0f : f;
    ei -= low ? 1 : 0;
    const float num = near_one ? -dn : m - 1.0f;
    const float den = near_one ? dd : m + 1.0f;
    const float t = num / den;
    const float e = near_one ? 0.0f : (float)ei;
    const float s = t * t;
    float p = atanh_coeff_f(kAtanhTermsF);
#pragma unroll
    for (int k = kAtanhTermsF - 1; k >= 0; --k) p = p * s + atanh_coeff_f(k);
    const float a = e * kLn2F;
    const float b = 2.0f * (t * p);
    return a + b;
}

__device__ __forceinline__ void bm_cos_sin_f(uint32_t w, float& cos_t, float& sin_t) {
#pragma clang fp contract(off)
    const uint32_t q = w >> 30;
    const uint32_t rho = w & 0x3FFFFFFFu;
    const bool direct = rho < (1u << 29);
    const uint32_t n = direct ? rho : (1u << 30) - rho;
    const float x = ((float)n * kTwoM32F) * kTwoPiF;
    const float z = x * x;
    float pc = cos_coeff_f(kCosTermsF);
#pragma unroll
    for (int k = kCosTermsF - 1; k >= 0; --k) pc = pc * z + cos_coeff_f(k);
    float ps = sin_coeff_f(kSinTermsF);
#pragma unroll
    for (int k = kSinTermsF - 1; k >= 0; --k) ps = ps * z + sin_coeff_f(k);
    const float c = pc, s = x * ps;
    // (cos, sin) of alpha, then the quadrant rotation: q odd swaps the pair,
    // cos changes sign for q = 1, 2 and sin for q = 2, 3 (exact)
    const float ca = direct ? c : s;
    const float sa = direct ? s : c;
    const float c0 = (q & 1u) ? sa : ca;
    const float s0 = (q & 1u) ? ca : sa;
    cos_t = (q == 1u || q == 2u) ? -c0 : c0;
    sin_t = (q >= 2u) ? -s0 : s0;
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& ga, float& gb) {
#pragma clang fp contract(off)
    const float r = sqrtf(-2.0f * bm_log_word_f(wa));
    float c, s;
    bm_cos_sin_f(wb, c, s);
    ga = r * c;
    gb = r * s;
}

// Deviates of cells 4g .. 4g+3 in the path's arithmetic type.
template <typename T>
__device__ __forceinline__ void noise_group(uint64_t g, uint64_t seed, uint32_t stream, T out[4]) {
    const u32x4 w = philox4x32_10({(uint32_t)g, (uint32_t)(g >> 32), stream, 0u}, (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    box_muller(w.x, w.y, out[0], out[1]);
    box_muller(w.z, w.w, out[2], out[3]);
}

}  // namespace gg
