"""Unit Gaussian deviates from Philox words (Box-Muller), defined operation by
operation so that any IEEE-754 binary64 implementation reproduces them bit for
bit.

The paper asks for white noise made of independent Gaussian numbers with zero
mean and unit variance (Sec. 2, step 1).  Library ``log``/``cos`` differ in
their last bit between platforms, so this module fixes its own elementary
functions built only from correctly rounded +, -, *, / and sqrt, exact
power-of-two scaling and exact integer manipulation, each result rounded once
in the order written below (no fused multiply-add).

Box-Muller (G. E. P. Box and M. E. Muller, Ann. Math. Stat. 29 (1958) 610):
from two uniforms u1 in (0, 1] and u2 in [0, 1),
    r = sqrt(-2 ln u1),  theta = 2 pi u2,  g_a = r cos theta,  g_b = r sin theta
are two independent N(0,1) deviates; the noise field keeps g_a only.

Uniforms from two 32-bit words (w_a, w_b):
    u1 = (w_a + 1) * 2^-32  (exact; never 0, so ln is finite)
    u2 = w_b * 2^-32        (exact)

ln(u1): write u1 = m * 2^e with m in [sqrt(1/2), sqrt(2)) (exact, via frexp
and one exact doubling); then ln u1 = e*LN2 + 2 atanh(t), t = (m-1)/(m+1),
and 2 atanh(t) = 2 t sum_{k=0..11} t^(2k)/(2k+1) (|t| <= 0.1716, so the first
omitted term is below 2e-20 relative).  The coefficients are 1/(2k+1),
each a single correctly rounded division.

cos/sin(2 pi u2): the top two bits of w_b give the quadrant q exactly; the
remaining 30 bits rho give the angle alpha = 2 pi rho 2^-32 in [0, pi/2).
If rho < 2^29, x = (rho 2^-32) * TWO_PI and (cos alpha, sin alpha) =
(C(x), S(x)); otherwise x = ((2^30 - rho) 2^-32) * TWO_PI (the reflected
angle pi/2 - alpha, formed from an exact integer) and (cos alpha, sin alpha) =
(S(x), C(x)).  Either way x lies in [0, pi/4].  C and S are the Taylor series
of cos and sin through x^16 and x^17 (first omitted term below 3e-18),
evaluated by Horner's rule in z = x*x with coefficients (-1)^k/(2k)! and
(-1)^k/(2k+1)! (factorials exact in binary64, one division each).  The
quadrant rotation (cos, sin) -> (-sin, cos) etc. only swaps and negates.

Pins (tests/test_oracle_noise.py): ln and the cos/sin pair agree with the
platform's libm to a few ulp over millions of arguments (a dropped series term
or a wrong coefficient would show at 1e-10 or worse); the deviates have the
moments and the distribution (Kolmogorov-Smirnov) of N(0,1); the reflected
branch joins the direct branch continuously at pi/4.
"""
import numpy as np

LN2 = 0.6931471805599453  # binary64 nearest to ln 2
TWO_PI = 6.283185307179586  # binary64 nearest to 2 pi
SQRT_HALF = 0.7071067811865476  # binary64 nearest to sqrt(1/2)
TWO_M32 = 2.0 ** -32

N_ATANH = 11  # highest power of t^2 kept in the atanh series
N_TRIG = 8    # highest power of z = x^2 kept in the cos and sin series


def _atanh_coeffs():
    return [1.0 / float(2 * k + 1) for k in range(N_ATANH + 1)]


def _factorial(n):
    f = 1.0
    for i in range(2, n + 1):
        f = f * float(i)  # exact: n! < 2^53 for n <= 18
    return f


def _cos_coeffs():
    return [(-1.0 if k % 2 else 1.0) / _factorial(2 * k) for k in range(N_TRIG + 1)]


def _sin_coeffs():
    return [(-1.0 if k % 2 else 1.0) / _factorial(2 * k + 1) for k in range(N_TRIG + 1)]


def log_unit(u):
    """ln(u) for binary64 u > 0, by the fixed operation sequence above."""
    u = np.asarray(u, dtype=np.float64)
    f, e = np.frexp(u)                     # u = f 2^e, f in [0.5, 1)
    low = f < SQRT_HALF
    m = np.where(low, f * 2.0, f)          # exact doubling
    e = np.where(low, e - 1, e).astype(np.float64)
    t = (m - 1.0) / (m + 1.0)
    s = t * t
    c = _atanh_coeffs()
    p = np.full_like(s, c[N_ATANH])
    for k in range(N_ATANH - 1, -1, -1):
        p = p * s + c[k]
    return e * LN2 + 2.0 * (t * p)


def _cos_sin_reduced(x):
    """Taylor cos and sin of x in [0, pi/4]."""
    z = x * x
    cc = _cos_coeffs()
    sc = _sin_coeffs()
    pc = np.full_like(z, cc[N_TRIG])
    ps = np.full_like(z, sc[N_TRIG])
    for k in range(N_TRIG - 1, -1, -1):
        pc = pc * z + cc[k]
        ps = ps * z + sc[k]
    return pc, x * ps


def cos_sin_turn(w):
    """(cos, sin) of 2 pi w 2^-32 for 32-bit integer words w."""
    w = np.asarray(w, dtype=np.uint64)
    q = (w >> np.uint64(30)).astype(np.int64)
    rho = (w & np.uint64((1 << 30) - 1)).astype(np.int64)
    direct = rho < (1 << 29)
    n = np.where(direct, rho, (1 << 30) - rho).astype(np.float64)   # exact
    x = (n * TWO_M32) * TWO_PI
    c, s = _cos_sin_reduced(x)
    ca = np.where(direct, c, s)
    sa = np.where(direct, s, c)
    cos_t = np.select([q == 0, q == 1, q == 2], [ca, -sa, -ca], sa)
    sin_t = np.select([q == 0, q == 1, q == 2], [sa, ca, -sa], -ca)
    return cos_t, sin_t


def box_muller(wa, wb):
    """The Box-Muller pair (g_a, g_b) = r (cos theta, sin theta) from two
    32-bit words each."""
    wa = np.asarray(wa, dtype=np.uint64)
    u1 = (wa + np.uint64(1)).astype(np.float64) * TWO_M32
    r = np.sqrt(-2.0 * log_unit(u1))
    cos_t, sin_t = cos_sin_turn(wb)
    return r * cos_t, r * sin_t


def gaussian(wa, wb):
    """One N(0,1) deviate per word pair: the cosine branch r cos(2 pi u2)."""
    return box_muller(wa, wb)[0]
