// Kernels of the initial-conditions path and their launchers, templated on
// the arithmetic type T (float or double).  Instantiated once per type in
// gg_f32.hip / gg_f64.hip.
//
// Data layouts (see include/gg.h): real fields row-major with axis 2
// contiguous; spectra as rows of complex values along k2.  The fused path
// keeps its spectra in a workspace whose rows hold only k2 in [0, N/2): the
// filter zeroes the k2 = N/2 Nyquist plane, so it is never stored.
//
// The five passes of the fused path (Sec. 2.1 Eq. (1)-(2), Sec. 2.2 Eq. (3)):
//   P1 noise + real-to-complex transform along axis 2       -> B0
//   P2 forward transform along axis 1                        B0 -> B0
//   P3 forward along axis 0, filter, two inverses along 0    B0 -> F (B0), G (B1)
//        F = IFFT_0(i s_0 tau W~),  G = IFFT_0(i tau W~)
//      (s_1 and s_2 are constant along an axis-0 line, so one inverse serves
//       both psi_1 = s_1 G and psi_2 = s_2 G)
//   P4 three inverses along axis 1                           F, G -> A (B0), C (B1), B (B2)
//        A = IFFT_1(F),  B = IFFT_1(s_1 G),  C = IFFT_1(G)
//   P5 complex-to-real along axis 2 of A, B, s_2 C + Eq. (3) -> positions, velocities
// tau[n^2] = (L / 2 pi) sqrt(P(k) N^3 / L^3) / (n^2 N^3) folds Eq. (1), the
// k_j/k^2 of Eq. (2) and the 1/N^3 of the inverse transform into one factor.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.h"
#include "noise_dev.h"

namespace gg {

// Plan data the kernels read (device pointers and scalars).
template <typename T>
struct PlanView {
    int n;
    double box;
    double cell;            // L / N (binary64)
    double offset;          // Lagrangian offset in cells
    double vfac;            // a H f
    const cx<T>* tw;        // tw[m] = exp(-2 pi i m / N), m < N
    const T* tau;           // tau[n^2], n^2 <= 3 (N/2)^2
};

// Signed mode index of k in [0, n).
__device__ __forceinline__ int signed_mode(int k, int n) { return k < (n >> 1) ? k : k - n; }

// ---------------------------------------------------------------------------
// White noise, four cells per thread.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_noise(T* __restrict__ w, uint64_t ngroups, uint64_t seed, uint32_t stream) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups;
         g += (uint64_t)gridDim.x * blockDim.x) {
        double d[4];
        noise_group(g, seed, stream, d);
        T* o = w + 4 * g;
        o[0] = (T)d[0];
        o[1] = (T)d[1];
        o[2] = (T)d[2];
        o[3] = (T)d[3];
    }
}

// ---------------------------------------------------------------------------
// P1 / forward axis-2 pass: L real lines of N points (from the noise
// generator or from memory) -> half spectra k2 in [0, N/2) (+ N/2 if NYQ).
// The N reals are packed as N/2 complex z[m] = x[2m] + i x[2m+1]; after the
// N/2-point transform Z, X[k] = E + W_N^k O with E = (Z[k] + conj Z[N/2-k])/2,
// O = (Z[k] - conj Z[N/2-k])/(2i); X[0] = Re Z0 + Im Z0, X[N/2] = Re Z0 - Im Z0.
// ---------------------------------------------------------------------------
template <typename T, int N, bool NOISE, bool NYQ>
__global__ __launch_bounds__(Tile<T>::L * PlanInfo<N / 2>::TPL) void k_zfwd(const T* __restrict__ in,
                                                                             cx<T>* __restrict__ out,
                                                                             const cx<T>* __restrict__ tw,
                                                                             uint64_t seed, uint32_t stream) {
    constexpr int M = N / 2;
    constexpr int L = Tile<T>::L;
    constexpr int TPL = PlanInfo<M>::TPL;
    constexpr int NT = L * TPL;
    constexpr int V = PlanInfo<M>::V;
    constexpr int MO = NYQ ? M + 1 : M;
    __shared__ cx<T> lds[L * M];
    const int t = threadIdx.x;
    const int c = t % L, j = t / L;
    const uint64_t line0 = (uint64_t)blockIdx.x * L;

    if constexpr (NOISE) {
        // group q of line cc covers cells 4q..4q+3 = complex slots 2q, 2q+1
        for (int gi = t; gi < L * (N / 4); gi += NT) {
            const int cc = gi % L, q = gi / L;
            double d[4];
            noise_group((line0 + cc) * (N / 4) + q, seed, stream, d);
            lds[lidx<L>(2 * q, cc)] = {(T)d[0], (T)d[1]};
            lds[lidx<L>(2 * q + 1, cc)] = {(T)d[2], (T)d[3]};
        }
    } else {
        const cx<T>* src = reinterpret_cast<const cx<T>*>(in + line0 * N);
        for (int fi = t; fi < L * M; fi += NT) {
            const int cc = fi / M, p = fi % M;
            lds[lidx<L>(p, cc)] = src[fi];
        }
    }
    __syncthreads();
    cx<T> v[V];
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = lds[lidx<L>(first_pos<M, -1>(j, i), c)];
    __syncthreads();
    fft_lines<T, M, L, -1, 2>(v, lds, tw, c, j);
#pragma unroll
    for (int i = 0; i < V; ++i) lds[lidx<L>(last_pos<M, -1>(j, i), c)] = v[i];
    __syncthreads();
    cx<T>* dst = out + line0 * MO;
    for (int fi = t; fi < L * MO; fi += NT) {
        const int cc = fi / MO, k = fi % MO;
        cx<T> x;
        if (k == 0 || k == M) {
            const cx<T> z0 = lds[lidx<L>(0, cc)];
            x = {k == 0 ? z0.x + z0.y : z0.x - z0.y, (T)0};
        } else {
            const cx<T> a = lds[lidx<L>(k, cc)];
            const cx<T> bz = lds[lidx<L>(M - k, cc)];
            const cx<T> b = {bz.x, -bz.y};
            const cx<T> e = cscale(cadd(a, b), (T)0.5);
            const cx<T> d = csub(a, b);
            const cx<T> o = {d.y * (T)0.5, -d.x * (T)0.5};
            x = cadd(e, cmul(o, tw[k]));
        }
        dst[fi] = x;
    }
}

// ---------------------------------------------------------------------------
// Eq. (3) for one value: position (sum in binary64, one wrap into [0, L),
// float rounding, L -> 0) and velocity a H f psi in the path's type.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void zel_point(T psi, int m, double cell, double offset, double box, T vfac, float& pos,
                                          float& vel) {
#pragma clang fp contract(off)
    const double q = ((double)m + offset) * cell;
    double x = q + (double)psi;
    if (x < 0.0) x = x + box;
    else if (x >= box) x = x - box;
    float xf = (float)x;
    if (xf >= (float)box) xf = 0.0f;
    pos = xf;
    vel = (float)(vfac * psi);
}

// ---------------------------------------------------------------------------
// P5 / inverse axis-2 pass: L half-spectrum lines -> real lines.  With the
// packing above run backwards: Z[k] = (X[k] + conj X[M-k]) +
// i W_N^-k (X[k] - conj X[M-k]) (Z[0] from the real parts of X[0], X[M]),
// an M-point inverse gives x[2m] + i x[2m+1] (unnormalised).
// MODE 0: write scale * x to a real field.  MODE 1: Eq. (3) for component
// blockIdx.y (whose spectrum is multiplied by s_2 = k when ZMUL).
// ---------------------------------------------------------------------------
struct ZelArgs {
    float* pos;
    float* vel;
    void* psi;  // optional displacement output (path type), may be null
};

template <typename T, int N, int MODE>
__global__ __launch_bounds__(Tile<T>::L * PlanInfo<N / 2>::TPL) void k_zinv(
    const cx<T>* __restrict__ in0, const cx<T>* __restrict__ in1, const cx<T>* __restrict__ in2, int istride,
    T* __restrict__ out, T scale, PlanView<T> pv, ZelArgs za) {
    constexpr int M = N / 2;
    constexpr int L = Tile<T>::L;
    constexpr int TPL = PlanInfo<M>::TPL;
    constexpr int NT = L * TPL;
    constexpr int V = PlanInfo<M>::V;
    __shared__ cx<T> lds[L * M];
    __shared__ T nyq[L];
    const int t = threadIdx.x;
    const int c = t % L, j = t / L;
    const uint64_t line0 = (uint64_t)blockIdx.x * L;
    const int comp = (MODE == 1) ? (int)blockIdx.y : 0;
    const cx<T>* in = comp == 0 ? in0 : (comp == 1 ? in1 : in2);
    const bool zmul = (MODE == 1) && comp == 2;
    const cx<T>* src = in + line0 * istride;
    for (int fi = t; fi < L * M; fi += NT) {
        const int cc = fi / M, k = fi % M;
        cx<T> x = src[(int64_t)cc * istride + k];
        if (zmul) x = cscale(x, (T)k);
        lds[lidx<L>(k, cc)] = x;
    }
    if (t < L) nyq[t] = (istride > M) ? src[(int64_t)t * istride + M].x : (T)0;
    __syncthreads();
    cx<T> v[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const int p = first_pos<M, 1>(j, i);
        const cx<T> xp = lds[lidx<L>(p, c)];
        if (p == 0) {
            const T a0 = xp.x, am = nyq[c];
            v[i] = {a0 + am, a0 - am};
        } else {
            const cx<T> xm = lds[lidx<L>(M - p, c)];
            const cx<T> b = {xm.x, -xm.y};
            const cx<T> s = cadd(xp, b);
            const cx<T> d = csub(xp, b);
            v[i] = cadd(s, mul_i(cmulc(d, pv.tw[p])));
        }
    }
    __syncthreads();
    fft_lines<T, M, L, 1, 2>(v, lds, pv.tw, c, j);
#pragma unroll
    for (int i = 0; i < V; ++i) lds[lidx<L>(last_pos<M, 1>(j, i), c)] = v[i];
    __syncthreads();
    const int n = N;
    const uint64_t n3 = (uint64_t)n * n * n;
    for (int fi = t; fi < L * M; fi += NT) {
        const int cc = fi / M, m = fi % M;
        const cx<T> z = lds[lidx<L>(m, cc)];
        const uint64_t line = line0 + cc;
        const uint64_t cell = line * N + 2 * m;
        if constexpr (MODE == 0) {
            *reinterpret_cast<cx<T>*>(out + cell) = {z.x * scale, z.y * scale};
        } else {
            const uint64_t off = (uint64_t)comp * n3 + cell;
            int m0, m1;
            if (comp == 0) m0 = m1 = (int)(line / N);
            else if (comp == 1) m0 = m1 = (int)(line % N);
            else { m0 = 2 * m; m1 = 2 * m + 1; }
            float p0, p1, u0, u1;
            zel_point<T>(z.x, m0, pv.cell, pv.offset, pv.box, (T)pv.vfac, p0, u0);
            zel_point<T>(z.y, m1, pv.cell, pv.offset, pv.box, (T)pv.vfac, p1, u1);
            *reinterpret_cast<float2*>(za.pos + off) = make_float2(p0, p1);
            *reinterpret_cast<float2*>(za.vel + off) = make_float2(u0, u1);
            if (za.psi) *reinterpret_cast<cx<T>*>(static_cast<T*>(za.psi) + off) = z;
        }
    }
}

// ---------------------------------------------------------------------------
// Strided passes: transforms of length N along an axis whose elements are
// pstride apart, for L contiguous columns at a time (one 128-byte row chunk
// per element).  Tile blockIdx.x -> (outer index o, column block).  Element
// (o, p, col) is at o * ostride + p * pstride + col.
//   SMODE_FWD / SMODE_INV : src -> dst (may alias), forward / unnormalised inverse
//   SMODE_XFILT (P3)      : axis 0 with o = k1, col = k2
//   SMODE_YINV3 (P4)      : axis 1 with o = m0, col = k2
// ---------------------------------------------------------------------------
enum { SMODE_FWD = 0, SMODE_INV = 1, SMODE_XFILT = 2, SMODE_YINV3 = 3 };

template <typename T>
struct StridedArgs {
    const cx<T>* src;
    cx<T>* dst0;
    cx<T>* dst1;
    cx<T>* dst2;
    int64_t ostride;
    int64_t pstride;
    int ncols;
    int ncb;  // column blocks per outer index
};

template <typename T, int N, int MODE>
__global__ __launch_bounds__(Tile<T>::L * PlanInfo<N>::TPL) void k_strided(StridedArgs<T> a, PlanView<T> pv) {
    constexpr int L = Tile<T>::L;
    constexpr int V = PlanInfo<N>::V;
    static_assert(PlanInfo<N>::template last_radix<-1>() == PlanInfo<N>::template first_radix<1>(),
                  "inverse plan must start where the forward plan ends");
    __shared__ cx<T> lds[L * N];
    const int t = threadIdx.x;
    const int c = t % L, j = t / L;
    const int o = blockIdx.x / a.ncb;
    const int col = (blockIdx.x % a.ncb) * L + c;
    const bool valid = col < a.ncols;
    const int64_t base = (int64_t)o * a.ostride + col;
    cx<T> v[V];

    if constexpr (MODE == SMODE_FWD || MODE == SMODE_INV) {
        constexpr int DIR = MODE == SMODE_FWD ? -1 : 1;
#pragma unroll
        for (int i = 0; i < V; ++i)
            v[i] = valid ? a.src[base + (int64_t)first_pos<N, DIR>(j, i) * a.pstride] : cx<T>{0, 0};
        fft_lines<T, N, L, DIR, 1>(v, lds, pv.tw, c, j);
        if (valid) {
#pragma unroll
            for (int i = 0; i < V; ++i) a.dst0[base + (int64_t)last_pos<N, DIR>(j, i) * a.pstride] = v[i];
        }
    } else if constexpr (MODE == SMODE_XFILT) {
#pragma unroll
        for (int i = 0; i < V; ++i)
            v[i] = valid ? a.src[base + (int64_t)first_pos<N, -1>(j, i) * a.pstride] : cx<T>{0, 0};
        fft_lines<T, N, L, -1, 1>(v, lds, pv.tw, c, j);
        // Eq. (1)-(2) on the spectrum held in registers (positions = axis-0 modes)
        const int s1 = signed_mode(o, N);
        const int s2 = col;
        const bool line_zero = (s1 == -(N / 2)) || (s2 >= N / 2);
        cx<T> g[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int k0 = last_pos<N, -1>(j, i);
            const int s0 = signed_mode(k0, N);
            const int n2 = s0 * s0 + s1 * s1 + s2 * s2;
            const bool zero = line_zero || (k0 == N / 2);
            const T tau = zero ? (T)0 : pv.tau[n2];  // tau[0] = 0 removes the mean
            const cx<T> it = mul_i(cscale(v[i], tau));
            g[i] = it;
            v[i] = cscale(it, (T)s0);
        }
        fft_lines<T, N, L, 1, 1>(v, lds, pv.tw, c, j);
        if (valid) {
#pragma unroll
            for (int i = 0; i < V; ++i) a.dst0[base + (int64_t)last_pos<N, 1>(j, i) * a.pstride] = v[i];
        }
        fft_lines<T, N, L, 1, 1>(g, lds, pv.tw, c, j);
        if (valid) {
#pragma unroll
            for (int i = 0; i < V; ++i) a.dst1[base + (int64_t)last_pos<N, 1>(j, i) * a.pstride] = g[i];
        }
    } else {  // SMODE_YINV3: src = F, dst1 = G (read, then C in place), dst0 = A (over F), dst2 = B
        cx<T> g[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int64_t off = base + (int64_t)first_pos<N, 1>(j, i) * a.pstride;
            v[i] = valid ? a.src[off] : cx<T>{0, 0};
            g[i] = valid ? a.dst1[off] : cx<T>{0, 0};
        }
        fft_lines<T, N, L, 1, 1>(v, lds, pv.tw, c, j);
        if (valid) {
#pragma unroll
            for (int i = 0; i < V; ++i) a.dst0[base + (int64_t)last_pos<N, 1>(j, i) * a.pstride] = v[i];
        }
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = cscale(g[i], (T)signed_mode(first_pos<N, 1>(j, i), N));
        fft_lines<T, N, L, 1, 1>(v, lds, pv.tw, c, j);
        if (valid) {
#pragma unroll
            for (int i = 0; i < V; ++i) a.dst2[base + (int64_t)last_pos<N, 1>(j, i) * a.pstride] = v[i];
        }
        fft_lines<T, N, L, 1, 1>(g, lds, pv.tw, c, j);
        if (valid) {
#pragma unroll
            for (int i = 0; i < V; ++i) a.dst1[base + (int64_t)last_pos<N, 1>(j, i) * a.pstride] = g[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Stand-alone Eq. (1)-(2) on a full half spectrum (k2 in [0, N/2]).
// tau here carries the 1/N^3 of the fused path; scale = N^3 removes it.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_filter(const cx<T>* __restrict__ w, cx<T>* __restrict__ psi, cx<T>* __restrict__ delta, int n,
                         T scale, T kf, const T* __restrict__ tau) {
    const int mo = n / 2 + 1;
    const uint64_t total = (uint64_t)n * n * mo;
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        const int k2 = (int)(idx % mo);
        const uint64_t r = idx / mo;
        const int k1 = (int)(r % n), k0 = (int)(r / n);
        const int s0 = signed_mode(k0, n), s1 = signed_mode(k1, n), s2 = k2;
        const int n2 = s0 * s0 + s1 * s1 + s2 * s2;
        const bool zero = (k0 == n / 2) || (k1 == n / 2) || (k2 == n / 2);
        const T ts = zero ? (T)0 : tau[n2] * scale;
        const cx<T> it = mul_i(cscale(w[idx], ts));
        psi[idx] = cscale(it, (T)s0);
        psi[total + idx] = cscale(it, (T)s1);
        psi[2 * total + idx] = cscale(it, (T)s2);
        if (delta) delta[idx] = cscale(w[idx], ts * (T)n2 * kf);
    }
}

// ---------------------------------------------------------------------------
// Stand-alone Eq. (3) over three displacement fields.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_zeldovich(const T* __restrict__ psi, float* __restrict__ pos, float* __restrict__ vel,
                            PlanView<T> pv) {
    const int n = pv.n;
    const uint64_t n3 = (uint64_t)n * n * n;
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < 3 * n3;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        const int comp = (int)(idx / n3);
        const uint64_t cell = idx % n3;
        int m;
        if (comp == 0) m = (int)(cell / ((uint64_t)n * n));
        else if (comp == 1) m = (int)((cell / n) % n);
        else m = (int)(cell % n);
        zel_point<T>(psi[idx], m, pv.cell, pv.offset, pv.box, (T)pv.vfac, pos[idx], vel[idx]);
    }
}

}  // namespace gg
