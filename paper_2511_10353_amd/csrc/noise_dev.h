// Device white noise: one Philox-4x32-10 call per cell -> one Box-Muller
// deviate in binary64.
//
// The paper's step 1 (Sec. 2) asks for independent unit Gaussians per cell and
// leaves the generator's mapping open.  Cell c is one Philox call with key =
// the 64-bit seed and counter = (c low word, c high word, stream, 0); of its
// words, w0 and w1 give g = sqrt(-2 ln u1) cos(2 pi u2) (the cosine branch of
// Box-Muller), u1 = (w0 + 1) 2^-32, u2 = w1 2^-32.  The float path stores g
// rounded once to float32.
//
// Philox-4x32 (Salmon, Moraes, Dror, Shaw, SC'11): per round, the 64-bit
// products M0*x0 and M1*x2 are split into high/low words and the state
// becomes (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0));
// the key advances by the Weyl constants after each round; 10 rounds.
//
// Box-Muller uses only correctly rounded +, -, *, /, sqrt and exact bit
// manipulation, in a fixed order with contraction disabled, so that any IEEE
// binary64 implementation of the same sequence gives the same bits:
//   ln u1 = e LN2 + 2 t P(t^2), u1 = m 2^e, m in [sqrt(1/2), sqrt(2)),
//           t = (m-1)/(m+1), P = sum_{k<=11} t^(2k)/(2k+1) (Horner)
//   cos(2 pi u2): quadrant from the top two bits, the 30-bit remainder
//           reflected about pi/4 by an exact integer subtraction, then the
//           Taylor series of cos (to x^16) or sin (to x^17) on [0, pi/4]
//           (Horner in x^2), coefficients (-1)^k/(2k)! and (-1)^k/(2k+1)!.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <type_traits>

namespace gg {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

struct u32x4 {
    uint32_t x, y, z, w;
};

template <int ROUNDS>
__device__ __forceinline__ u32x4 philox_rounds(u32x4 ctr, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        // one 32x32 -> 64-bit product per multiplier gives both halves; the
        // three-input XORs are single v_bitop3 instructions (truth table 0x96)
        const uint64_t p0 = (uint64_t)kPhiloxM0 * ctr.x;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * ctr.z;
        uint32_t a, b;
        asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(a) : "v"((uint32_t)(p1 >> 32)), "v"(ctr.y), "s"(k0));
        asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(b) : "v"((uint32_t)(p0 >> 32)), "v"(ctr.w), "s"(k1));
        ctr = {a, (uint32_t)p1, b, (uint32_t)p0};
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return ctr;
}

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 ctr, uint32_t k0, uint32_t k1) {
    return philox_rounds<10>(ctr, k0, k1);
}

// Philox-4x32-10 of the counter (c, 0, stream, 0), the same function with its
// first two rounds written out: the words that depend only on the key and the
// stream (the first after round one, the last after round two) and the
// product between them stay wave-uniform, in scalar registers.
__device__ __forceinline__ u32x4 philox4x32_10_c32(uint32_t c, uint32_t stream, uint32_t k0, uint32_t k1) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * stream;
    const uint32_t x0 = (uint32_t)(p1 >> 32) ^ k0;  // the counter's words 1 and 3 are 0
    const uint32_t x1 = (uint32_t)p1;
    const uint32_t x2 = (uint32_t)(p0 >> 32) ^ k1;
    const uint32_t x3 = (uint32_t)p0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    const uint64_t q0 = (uint64_t)kPhiloxM0 * x0;
    const uint64_t q1 = (uint64_t)kPhiloxM1 * x2;
    const u32x4 ctr = {(uint32_t)(q1 >> 32) ^ x1 ^ k0, (uint32_t)q1, (uint32_t)(q0 >> 32) ^ x3 ^ k1, (uint32_t)q0};
    return philox_rounds<8>(ctr, k0 + kPhiloxW0, k1 + kPhiloxW1);
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

// cos(2 pi w 2^-32): with alpha = 2 pi rho 2^-32 the remainder angle of the
// quadrant q, cos(q pi/2 + alpha) is cos alpha, -sin alpha, -cos alpha,
// sin alpha for q = 0..3; cos alpha = C(x), sin alpha = S(x) when rho < 2^29
// (x = alpha), and the other way round after reflection (x = pi/2 - alpha).
// Both series are evaluated (straight-line code, no per-term selects) and
// the one the quadrant and reflection call for is kept.
__device__ __forceinline__ double bm_cos(uint32_t w) {
#pragma clang fp contract(off)
    const uint32_t q = w >> 30;
    const uint32_t rho = w & 0x3FFFFFFFu;
    const bool direct = rho < (1u << 29);
    const uint32_t n = direct ? rho : (1u << 30) - rho;
    const double x = ((double)n * kTwoM32) * kTwoPi;
    const double z = x * x;
    const bool use_cos = ((q & 1u) == 0u) == direct;
    double pc = cos_coeff(kTrigTerms), ps = sin_coeff(kTrigTerms);
#pragma unroll
    for (int k = kTrigTerms - 1; k >= 0; --k) {
        pc = pc * z + cos_coeff(k);
        ps = ps * z + sin_coeff(k);
    }
    const double v = use_cos ? pc : x * ps;
    return (q == 1u || q == 2u) ? -v : v;
}

// The binary64 deviate of a cell from its words w0, w1.
__device__ __forceinline__ double gaussian_words(uint32_t w0, uint32_t w1) {
#pragma clang fp contract(off)
    const double u1 = (double)((uint64_t)w0 + 1ull) * kTwoM32;
    const double r = sqrt(-2.0 * bm_log(u1));
    return r * bm_cos(w1);
}

__device__ __forceinline__ u32x4 cell_words(uint64_t c, uint64_t seed, uint32_t stream) {
    return philox4x32_10({(uint32_t)c, (uint32_t)(c >> 32), stream, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// The binary64 deviate of cell c.
__device__ __forceinline__ double gaussian_cell(uint64_t c, uint64_t seed, uint32_t stream) {
    const u32x4 w = cell_words(c, seed, stream);
    return gaussian_words(w.x, w.y);
}

// Logarithm table of the float path.  With z0 the double whose bits are
// kLnTabLoBits (about 0.709), a positive double u is written u = 2^k z with z
// in [z0, 2 z0) by integer arithmetic on its bits: t = bits(u) - kLnTabLoBits,
// k = t >> 52 (arithmetic), bits(z) = bits(u) - k 2^52.  Bits 45..51 of t select one of
// 128 buckets of z, equal in bit space (2^-8 wide below 1, 2^-7 above).
// Entry i is (invc, 2 ln invc) for an inverse centre invc of bucket i, so
// that ln u = k ln 2 - ln invc + ln(1 + r) with r = z invc - 1, |r| < 2^-8.
// z0 is placed so that 1 lies in the middle of its bucket, whose entry
// is (1, 0): near u = 1 the logarithm is ln(1 + r) with r = z - 1 exact, and
// next to that bucket |ln z| > 2^-9.5, so the cancellation of 2 ln invc
// against 2 ln(1 + r) costs at most a factor of about 2.
constexpr int kLnTabBits = 7;
constexpr int kLnTab = 1 << kLnTabBits;
constexpr uint64_t kLnTabLoBits = 0x3FF0000000000000ull - (uint64_t)(2 * 74 + 1) * (1ull << (51 - kLnTabBits));

// Host side: fills t[0 .. kLnTab) (x = invc, y = 2 ln invc).  invc is the
// reciprocal of the bucket's midpoint in value; the logarithm comes from the
// host's libm (within an ulp or so), far inside the float path's 2^-46.
inline void make_ln_table(double2* t) {
    const uint64_t one = 0x3FF0000000000000ull;
    for (int i = 0; i < kLnTab; ++i) {
        const uint64_t lo = kLnTabLoBits + ((uint64_t)i << (52 - kLnTabBits));
        const uint64_t hi = lo + (1ull << (52 - kLnTabBits));
        double zlo, zhi;
        std::memcpy(&zlo, &lo, sizeof zlo);
        std::memcpy(&zhi, &hi, sizeof zhi);
        const double invc = (lo <= one && one < hi) ? 1.0 : 2.0 / (zlo + zhi);
        t[i] = make_double2(invc, 2.0 * std::log(invc));
    }
}

// The same deviate to about 2^-46 relative, for the float path: -2 ln u1
// from the table above and ln(1 + r) to r^6 (truncation below 2^-50 of the
// result, also next to the bucket of 1), the square root by a reciprocal
// square root estimate and one Goldschmidt step, and cos(2 pi u2) as
// +-sin(2 pi n 2^-32) with n in [0, 2^30] (cos(alpha) = sin(pi/2 - alpha)
// taken on the integer angle, so one odd Taylor series to x^19 covers every
// quadrant; truncation below 2^-51 on [0, pi/2]).  The hardware estimate is
// good to about 2^-24, so the refinement leaves about 2^-47.  u1 is the exact
// value the defining sequence forms; r = -0 when -2 ln u1 = 0, as sqrt(-0)
// gives there.  lnt: the table, in LDS.
__device__ __forceinline__ double gaussian_words_fast(uint32_t w0, uint32_t w1, const double2* lnt) {
    const double u1 = fma((double)w0, kTwoM32, kTwoM32);  // (w0 + 1) 2^-32, exact
    const uint64_t ix = (uint64_t)__double_as_longlong(u1);
    const uint64_t tb = ix - kLnTabLoBits;
    const int k = (int)((int64_t)tb >> 52);
    const double2 ent = lnt[(uint32_t)(tb >> (52 - kLnTabBits)) & (kLnTab - 1)];
    const double z = __longlong_as_double((long long)(ix - ((uint64_t)(int64_t)k << 52)));
    const double r0 = fma(z, ent.x, -1.0);
    double p = fma(r0, 1.0 / 6.0, -1.0 / 5.0);
    p = fma(p, r0, 1.0 / 4.0);
    p = fma(p, r0, -1.0 / 3.0);
    p = fma(p, r0, 1.0 / 2.0);
    const double lp = fma(-(r0 * r0), p, r0);  // ln(1 + r0)
    const double a = fma(lp, -2.0, fma((double)k, -2.0 * kLn2, ent.y));  // -2 ln u1 >= 0
    const double y = __builtin_amdgcn_rsq(a);
    const double g0 = a * y, h0 = 0.5 * y;
    const double rr = fma(-g0, h0, 0.5);
    const double r = a > 0.0 ? fma(g0, rr, g0) : -0.0;
    const uint32_t q = w1 >> 30;
    const uint32_t rho = w1 & 0x3FFFFFFFu;
    const uint32_t n = (q & 1u) ? rho : (1u << 30) - rho;
    const double x = (double)n * (kTwoPi * kTwoM32);
    const double zz = x * x;
    double ps = sin_coeff(9);
#pragma unroll
    for (int j = 8; j >= 0; --j) ps = fma(ps, zz, sin_coeff(j));
    const double v = x * ps;
    return r * ((q == 1u || q == 2u) ? -v : v);
}

// Cell c's deviate in the path's type: binary64 as defined above, or that
// value rounded once to float.  The float case rounds the fast evaluation g
// when every value within 2^-42 |g| of it rounds to the same float, and
// evaluates the defining sequence otherwise (about one cell in 10^5); the
// exact deviate lies within 2^-46 |g| of g.  The test works on the bits of
// g: a float rounding boundary of a normal double lies where its 29 low
// mantissa bits read 2^28, and 2^-42 |g| is below 2^11 units in the last
// place of g, so g is safe when those bits are more than 2^11 from 2^28
// (|g| > 2^-46 or g = 0 always, so float subnormals do not arise).
// lnt: the float path's logarithm table in LDS (unused by the double path).
template <typename T>
__device__ __forceinline__ T noise_of_words(const u32x4& w, const double2* lnt) {
    if constexpr (std::is_same_v<T, float>) {
        const double g = gaussian_words_fast(w.x, w.y, lnt);
        const uint32_t lo29 = (uint32_t)__double_as_longlong(g) & 0x1FFFFFFFu;
        if (__builtin_expect(lo29 - 0x10000000u + 2048u > 4096u, 1)) return (float)g;
        return (float)gaussian_words(w.x, w.y);
    } else {
        return gaussian_words(w.x, w.y);
    }
}

template <typename T>
__device__ __forceinline__ T noise_value(uint64_t c, uint64_t seed, uint32_t stream, const double2* lnt) {
    return noise_of_words<T>(cell_words(c, seed, stream), lnt);
}

// The same for a cell index below 2^32 (every lattice here has at most 2^30
// cells): the counter's high word is 0, so part of the first two rounds
// depends only on the seed and the stream (philox4x32_10_c32).
template <typename T>
__device__ __forceinline__ T noise_value32(uint32_t c, uint64_t seed, uint32_t stream, const double2* lnt) {
    return noise_of_words<T>(philox4x32_10_c32(c, stream, (uint32_t)seed, (uint32_t)(seed >> 32)), lnt);
}

}  // namespace gg
