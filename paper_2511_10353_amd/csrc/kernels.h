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

#include <type_traits>

#include "cosmo_dev.h"
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
    const T* tau;           // tau[n^2], n^2 <= 3 (N/2)^2, binary64 values rounded to T
    const float4* tauseg;   // piecewise-cubic tau (kTauSeg segments), float plans only
    const double2* tauseg64;  // piecewise degree-7 tau (kTauSeg64 x 4 double2), double plans only
    const double2* lntab;   // logarithm table of the noise (kLnTab entries), float plans only
    double amp_scale;       // displacement scale sqrt(A'/A) (1 for the plan's amplitude)
    // mode window of the axis-0 filter passes (Eq. 4-5): modes with
    // n2 < n2_lo or n2 >= n2_hi are dropped; deconv divides by the
    // cloud-in-cell window prod_j sinc^2(pi s_j / N)
    int n2_lo;
    int n2_hi;
    int deconv;
    // particle lattice q_j = origin[j] + (m_j + offset) cell, wrapped into
    // [0, wrap): a zoom level's sub-box inside the base box (origin 0 and
    // wrap = box for a full box)
    double origin[3];
    double wrap;
};

// 1 / sinc^2(pi s / N), the inverse of one axis of the cloud-in-cell window
template <typename T>
__device__ inline T cic_deconv(int s, int n) {
    if (s == 0) return (T)1;
    const double x = 3.14159265358979323846 * (double)s / (double)n;
    if constexpr (std::is_same_v<T, float>) {
        const float xf = (float)x, r = xf / sinf(xf);
        return r * r;
    } else {
        const double r = x / sin(x);
        return r * r;
    }
}

// The filter factor tau(n2) inside the axis-0 passes of the fused path.  The
// single-precision passes copy the piecewise-cubic table (15 KB) into LDS once
// per work-group and evaluate it (scattered reads of the full table missed
// the L1 and loaded L2 with one request per element); double precision reads
// the exact table.
template <typename T>
struct TauLookup {
    const T* tau;
    __device__ T operator()(int n2) const { return tau[n2]; }
};

template <>
struct TauLookup<double> {
    const double2* seg;
    __device__ double operator()(int n2) const {
        const uint32_t u = (uint32_t)n2;
        const int e = 31 - __clz(u | 1u);
        const int sh = e > 5 ? e - 5 : 0;
        const double2* c = seg + 4 * ((sh << 5) + (u >> sh));
        const double t = (double)(u & ((1u << sh) - 1u)) * __longlong_as_double((long long)(1023 - sh) << 52);
        const double2 c01 = c[0], c23 = c[1], c45 = c[2], c67 = c[3];
        double p = fma(t, c67.y, c67.x);
        p = fma(t, p, c45.y);
        p = fma(t, p, c45.x);
        p = fma(t, p, c23.y);
        p = fma(t, p, c23.x);
        p = fma(t, p, c01.y);
        return fma(t, p, c01.x);
    }
};

template <>
struct TauLookup<float> {
    const float4* seg;
    __device__ float operator()(int n2) const {
        const uint32_t u = (uint32_t)n2;
        const int e = 31 - __clz(u | 1u);
        const int sh = e > 6 ? e - 6 : 0;
        const float4 c = seg[(sh << 6) + (u >> sh)];
        const float t = (float)(u & ((1u << sh) - 1u)) * __int_as_float((127 - sh) << 23);
        return fmaf(t, fmaf(t, fmaf(t, c.w, c.z), c.y), c.x);
    }
};

// Call from every thread of the work-group before the first lookup; the
// caller's next __syncthreads() publishes the LDS copy.
template <typename T>
__device__ inline TauLookup<T> tau_lookup(const PlanView<T>& pv) {
    if constexpr (std::is_same_v<T, float>) {
        __shared__ float4 tl[kTauSeg];
        for (int i = threadIdx.x; i < kTauSeg; i += blockDim.x) tl[i] = pv.tauseg[i];
        return TauLookup<float>{tl};
    } else {
        __shared__ double2 tl[4 * kTauSeg64];
        for (int i = threadIdx.x; i < 4 * kTauSeg64; i += blockDim.x) tl[i] = pv.tauseg64[i];
        return TauLookup<double>{tl};
    }
}

// Returns x unchanged but hides its value from the optimiser, so that
// quantities derived from it inside a loop body are recomputed per iteration
// instead of being hoisted and kept live across the loop (register pressure).
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Signed mode index of k in [0, n).
__device__ __forceinline__ int signed_mode(int k, int n) { return k < (n >> 1) ? k : k - n; }

// ---------------------------------------------------------------------------
// White noise, one cell per thread and iteration.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_noise(T* __restrict__ w, uint64_t ncells, uint64_t seed, uint32_t stream, const double2* lntab) {
    const double2* lnt = nullptr;
    if constexpr (std::is_same_v<T, float>) {
        __shared__ double2 lt[kLnTab];
        for (int i = threadIdx.x; i < kLnTab; i += blockDim.x) lt[i] = lntab[i];
        __syncthreads();
        lnt = lt;
    }
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncells;
         c += (uint64_t)gridDim.x * blockDim.x)
        w[c] = noise_value<T>(c, seed, stream, lnt);
}

// Lattice coordinates (m0, m1) of spectrum row r.  Plain rows are r = m0 N + m1;
// the fused path's blocked rows are r = ((m0 / 8) N + m1) 8 + m0 % 8.
template <bool BLK>
__device__ __forceinline__ void row_coords(uint64_t r, int n, int& m0, int& m1) {
    if constexpr (BLK) {
        const uint64_t h = r >> 3;
        m0 = (int)((h / n) * 8 + (r & 7));
        m1 = (int)(h % n);
    } else {
        m0 = (int)(r / n);
        m1 = (int)(r % n);
    }
}

// ---------------------------------------------------------------------------
// P1 / forward axis-2 pass: L real lines of N points (from the noise
// generator or from memory) -> half spectra k2 in [0, N/2) (+ N/2 if NYQ).
// The N reals are packed as N/2 complex z[m] = x[2m] + i x[2m+1]; after the
// N/2-point transform Z, X[k] = E + W_N^k O with E = (Z[k] + conj Z[N/2-k])/2,
// O = (Z[k] - conj Z[N/2-k])/(2i); X[0] = Re Z0 + Im Z0, X[N/2] = Re Z0 - Im Z0.
// Block b handles rows row0 + b L + r, r < L (contiguous).
// ---------------------------------------------------------------------------
// Sum of one double per thread over a work-group of NT threads, written by
// thread 0 to *out.  Fixed order: butterfly within each wave, then the waves
// in index order (the result does not depend on scheduling).
template <int NT>
__device__ inline void block_sum(double v, double* out) {
    constexpr int W = NT < 64 ? NT : 64;
    constexpr int NW = NT / W;
    __shared__ double wsum[NW];
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    const int t = threadIdx.x;
    if (t % W == 0) wsum[t / W] = v;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < NW; ++i) s += wsum[i];
        *out = s;
    }
}

// Sources of the real lines of an axis-2 forward pass.
enum { ZSRC_NOISE = 0, ZSRC_REAL = 1, ZSRC_GRAD = 2 };

// ZSRC_REAL: lines of the real field w (plain rows, line (m0, m1) at
// (m0 N + m1) N).  ZSRC_GRAD: component blockIdx.y of the adjoint input
// g = gpsi + gpos + vfac gvel (any of the three may be null; 3 N^3 values each),
// written to out + blockIdx.y * ostride_comp.  If psi is not null, each block
// also writes sum g psi over its cells (g formed in binary64) to
// part[blockIdx.y gridDim.x + blockIdx.x], summed in a fixed order.
template <typename T>
struct ZSrc {
    const T* w;
    const T* gpsi;
    const float* gpos;
    const float* gvel;
    double vfac;
    uint64_t ostride_comp;
    const T* psi;
    double* part;
    // ZSRC_REAL with several fields: field blockIdx.y at w + blockIdx.y
    // wstride_comp.  kout > 0 (plain rows, no Nyquist column): only modes
    // k2 < kout are written, kout per line (a pruned half spectrum)
    uint64_t wstride_comp;
    int kout;
    // ZSRC_NOISE of float plans: the logarithm table of the noise
    const double2* lntab = nullptr;
};

template <typename T, int N, int SRC, bool NYQ, bool BLK, int L = Tile<T>::L>
__global__ __launch_bounds__(L * PlanInfo<N / 2>::TPL) void k_zfwd(ZSrc<T> zs, cx<T>* __restrict__ out,
                                                                             const cx<T>* __restrict__ tw,
                                                                             uint64_t seed, uint32_t stream,
                                                                             uint64_t row0) {
    constexpr int M = N / 2;
    constexpr int TPL = PlanInfo<M>::TPL;
    constexpr int NT = L * TPL;
    constexpr int V = PlanInfo<M>::V;
    constexpr int MO = NYQ ? M + 1 : M;
    __shared__ cx<T> lds[L * M];
    const int t = threadIdx.x;
    const int c = t % L, j = t / L;
    const uint64_t line0 = row0 + (uint64_t)blockIdx.x * L;

    cx<T> v[V];
    if constexpr (SRC == ZSRC_NOISE) {
        const double2* lnt = nullptr;
        if constexpr (std::is_same_v<T, float>) {
            __shared__ double2 lt[kLnTab];
            for (int i = t; i < kLnTab; i += NT) lt[i] = zs.lntab[i];
            __syncthreads();
            lnt = lt;
        }
        // complex slot p of a line holds cells 2p, 2p+1; each thread draws the
        // slots its first transform stage takes, so the tile is not staged
        // through LDS
        static_assert((uint64_t)N * N * N <= (1ull << 32), "cell indices are 32-bit");
        int m0, m1;
        row_coords<BLK>(line0 + c, N, m0, m1);
        const uint32_t base = ((uint32_t)m0 * N + (uint32_t)m1) * N;
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const uint32_t cell = base + 2u * (uint32_t)first_pos<M, -1>(j, i);
            v[i] = {noise_value32<T>(cell, seed, stream, lnt), noise_value32<T>(cell + 1, seed, stream, lnt)};
        }
    } else {
        // four consecutive reals (two packed complex slots) per lane
        double dacc = 0.0;
        const int comp = SRC == ZSRC_GRAD ? (int)blockIdx.y : 0;
        const uint64_t coff = (uint64_t)comp * N * N * N;
        for (int fi = t; fi < L * M / 2; fi += NT) {
            const int cc = fi / (M / 2), p = 2 * (fi % (M / 2));
            int m0, m1;
            row_coords<BLK>(line0 + cc, N, m0, m1);
            const uint64_t cell = ((uint64_t)m0 * N + m1) * N + 2 * p;
            cx<T> x0, x1;
            if constexpr (SRC == ZSRC_REAL) {
                const T* wsrc = zs.w + (uint64_t)blockIdx.y * zs.wstride_comp;
                x0 = *reinterpret_cast<const cx<T>*>(wsrc + cell);
                x1 = *reinterpret_cast<const cx<T>*>(wsrc + cell + 2);
            } else {
                T a[4] = {(T)0, (T)0, (T)0, (T)0};
                float4 b = {0.f, 0.f, 0.f, 0.f}, d = {0.f, 0.f, 0.f, 0.f};
                if (zs.gpsi) {
                    const T* q = zs.gpsi + coff + cell;
#pragma unroll
                    for (int e = 0; e < 4; ++e) a[e] = q[e];
                }
                if (zs.gpos) b = *reinterpret_cast<const float4*>(zs.gpos + coff + cell);
                if (zs.gvel) d = *reinterpret_cast<const float4*>(zs.gvel + coff + cell);
                const float bb[4] = {b.x, b.y, b.z, b.w}, dd[4] = {d.x, d.y, d.z, d.w};
                T g[4];
                const T vf = (T)zs.vfac;
#pragma unroll
                for (int e = 0; e < 4; ++e) g[e] = a[e] + (T)bb[e] + vf * (T)dd[e];
                if (zs.psi) {
                    const T* q = zs.psi + coff + cell;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        dacc += ((double)a[e] + (double)bb[e] + zs.vfac * (double)dd[e]) * (double)q[e];
                }
                x0 = {g[0], g[1]};
                x1 = {g[2], g[3]};
            }
            lds[lidx<L>(p, cc)] = x0;
            lds[lidx<L>(p + 1, cc)] = x1;
        }
        out += (uint64_t)blockIdx.y * zs.ostride_comp;
        if constexpr (SRC == ZSRC_GRAD) {
            if (zs.part) block_sum<NT>(dacc, zs.part + (uint64_t)blockIdx.y * gridDim.x + blockIdx.x);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = lds[lidx<L>(first_pos<M, -1>(j, i), c)];
        __syncthreads();
    }
    fft_lines<T, M, L, -1, 2>(v, lds, tw, c, j);
#pragma unroll
    for (int i = 0; i < V; ++i) lds[lidx<L>(last_pos<M, -1>(j, i), c)] = v[i];
    __syncthreads();
    auto post = [&](int cc, int k) -> cx<T> {
        if (k == 0 || k == M) {
            const cx<T> z0 = lds[lidx<L>(0, cc)];
            return {k == 0 ? z0.x + z0.y : z0.x - z0.y, (T)0};
        }
        const cx<T> a = lds[lidx<L>(k, cc)];
        const cx<T> bz = lds[lidx<L>(M - k, cc)];
        const cx<T> b = {bz.x, -bz.y};
        const cx<T> e = cscale(cadd(a, b), (T)0.5);
        const cx<T> d = csub(a, b);
        const cx<T> o = {d.y * (T)0.5, -d.x * (T)0.5};
        return cadd(e, cmul(o, tw[k]));
    };
    if constexpr (!NYQ && !BLK && SRC == ZSRC_REAL) {
        if (zs.kout > 0) {
            cx<T>* dk = out + line0 * zs.kout;
            for (int fi = t; fi < L * zs.kout; fi += NT) dk[fi] = post(fi / zs.kout, fi % zs.kout);
            return;
        }
    }
    cx<T>* dst = out + line0 * MO;
    if constexpr (NYQ) {
        for (int fi = t; fi < L * MO; fi += NT) dst[fi] = post(fi / MO, fi % MO);
    } else {
        for (int fi = t; fi < L * M / 2; fi += NT) {
            const int cc = fi / (M / 2), k = 2 * (fi % (M / 2));
            const cx<T> x0 = post(cc, k), x1 = post(cc, k + 1);
            dst[2 * fi] = x0;
            dst[2 * fi + 1] = x1;
        }
    }
}

// ---------------------------------------------------------------------------
// Eq. (3) for one value: position (sum in binary64, periodic image in [0, L),
// float rounding, L -> 0) and velocity a H f psi in the path's type.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void zel_point(T psi, int m, double origin, double cell, double offset, double box, T vfac,
                                          float& pos, float& vel) {
#pragma clang fp contract(off)
    const double q = origin + ((double)m + offset) * cell;
    double x = q + (double)psi;
    if (x < 0.0 || x >= box) {
        // periodic image x - L floor(x/L); the rounded quotient can leave the
        // result on L or just below 0, which one more period corrects
        x = x - box * floor(x / box);
        if (x < 0.0) x = x + box;
        else if (x >= box) x = x - box;
    }
    float xf = (float)x;
    if (xf >= (float)box) xf = 0.0f;
    pos = xf;
    vel = (float)(vfac * psi);
}

// ---------------------------------------------------------------------------
// Inverse axis-2 pass: L half-spectrum lines -> real lines.  With the packing
// above run backwards: Z[k] = (X[k] + conj X[M-k]) + i W_N^-k (X[k] - conj
// X[M-k]) (Z[0] from the real parts of X[0], X[M]), an M-point inverse gives
// x[2m] + i x[2m+1] (unnormalised).  Writes scale * x to a real field (plain
// rows); the input rows are plain or blocked as BLK says.
// ---------------------------------------------------------------------------

// Z[p] of the packing from the LDS tile (X[M] of every line is nyq[c]).
template <typename T, int M, int L>
__device__ __forceinline__ cx<T> c2r_pack(const cx<T>* lds, const cx<T>* tw, T nyq, int p, int c) {
    const cx<T> xp = lds[lidx<L>(p, c)];
    if (p == 0) {
        const T a0 = xp.x;
        return {a0 + nyq, a0 - nyq};
    }
    const cx<T> xm = lds[lidx<L>(M - p, c)];
    const cx<T> b = {xm.x, -xm.y};
    const cx<T> s = cadd(xp, b);
    const cx<T> d = csub(xp, b);
    return cadd(s, mul_i(cmulc(d, tw[p])));
}

template <typename T, int N, bool BLK, int L = Tile<T>::L>
__global__ __launch_bounds__(L * PlanInfo<N / 2>::TPL) void k_zinv(const cx<T>* __restrict__ in, int istride,
                                                                   int kin, uint64_t icomp, T* __restrict__ out,
                                                                   T scale, PlanView<T> pv, int kmul_field = -1) {
    constexpr int M = N / 2;
    constexpr int TPL = PlanInfo<M>::TPL;
    constexpr int NT = L * TPL;
    constexpr int V = PlanInfo<M>::V;
    __shared__ cx<T> lds[L * M];
    __shared__ T nyq[L];
    const int t = threadIdx.x;
    const int c = t % L, j = t / L;
    const uint64_t line0 = (uint64_t)blockIdx.x * L;
    const cx<T>* src = in + (uint64_t)blockIdx.y * icomp + line0 * istride;
    out += (uint64_t)blockIdx.y * N * N * N;
    if (istride == M && kin == M) {
        for (int fi = t; fi < L * M / 2; fi += NT) {
            const int cc = fi / (M / 2), k = 2 * (fi % (M / 2));
            lds[lidx<L>(k, cc)] = src[2 * fi];
            lds[lidx<L>(k + 1, cc)] = src[2 * fi + 1];
        }
        if (t < L) nyq[t] = (T)0;
    } else {
        // rows of istride modes of which the first kin are stored (kin = M + 1:
        // the full half spectrum; kin <= M: a pruned one, the rest zero)
        // field kmul_field (a displacement's third component) is multiplied by
        // its mode index k2, as the particle pass does
        const bool kmul = (int)blockIdx.y == kmul_field;
        for (int fi = t; fi < L * M; fi += NT) {
            const int cc = fi / M, k = fi % M;
            const cx<T> x = k < kin ? src[(int64_t)cc * istride + k] : cx<T>{(T)0, (T)0};
            lds[lidx<L>(k, cc)] = kmul ? cscale(x, (T)k) : x;
        }
        if (t < L) nyq[t] = kin > M ? src[(int64_t)t * istride + M].x : (T)0;
    }
    __syncthreads();
    cx<T> v[V];
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = c2r_pack<T, M, L>(lds, pv.tw, nyq[c], first_pos<M, 1>(j, i), c);
    __syncthreads();
    fft_lines<T, M, L, 1, 2>(v, lds, pv.tw, c, j);
#pragma unroll
    for (int i = 0; i < V; ++i) lds[lidx<L>(last_pos<M, 1>(j, i), c)] = v[i];
    __syncthreads();
    // four consecutive reals (two complex slots) per lane
    for (int fi = t; fi < L * M / 2; fi += NT) {
        const int cc = fi / (M / 2), m = 2 * (fi % (M / 2));
        const cx<T> z0 = lds[lidx<L>(m, cc)], z1 = lds[lidx<L>(m + 1, cc)];
        int m0, m1;
        row_coords<BLK>(line0 + cc, N, m0, m1);
        T* o = out + ((uint64_t)m0 * N + m1) * N + 2 * m;
        *reinterpret_cast<cx<T>*>(o) = {z0.x * scale, z0.y * scale};
        *reinterpret_cast<cx<T>*>(o + 2) = {z1.x * scale, z1.y * scale};
    }
}

// ---------------------------------------------------------------------------
// P5: the inverse axis-2 pass of the three displacement spectra (blocked rows,
// k2 < M; the Nyquist plane is zero) fused with Eq. (3).  A tile is L lines
// of one component; component 2's spectrum is multiplied by s_2 = k on the
// way into LDS (its tau carries no s_2).  PV: write positions and
// velocities; PS: write the displacements in the path's type.
//
// The grid is smaller than the tile count: work-group b takes every G-th tile
// of its range (G = gridDim.x / 8 and the range its XCD's eighth of the
// tiles when the grid is a multiple of 8, else G = gridDim.x over all
// tiles).  As soon as a tile sits in LDS, each thread loads its share of the
// next tile into registers, so those HBM reads run under the current tile's
// transform and stores.  The N-point twiddle table
// is copied into LDS once per work-group, so that the loop issues no other
// global load (loads complete in order: waiting for a later one would wait
// for the prefetch too).  The prefetch after the last tile re-reads that
// tile.
// ---------------------------------------------------------------------------
struct ZelArgs {
    float* pos;
    float* vel;
    void* psi;
};

template <typename T, int N, int L, bool PV, bool PS>
__global__ __launch_bounds__(L * PlanInfo<N / 2>::TPL) void k_zel(const cx<T>* __restrict__ in0,
                                                                  const cx<T>* __restrict__ in1,
                                                                  const cx<T>* __restrict__ in2, PlanView<T> pv,
                                                                  ZelArgs za, int ntiles) {
    constexpr int M = N / 2;
    constexpr int TPL = PlanInfo<M>::TPL;
    constexpr int NT = L * TPL;
    constexpr int V = PlanInfo<M>::V;
    constexpr int NF = L * M / 2 / NT;  // pairs of complex values per thread and tile
    static_assert(NF * NT == L * M / 2, "a tile is whole pairs per thread");
    constexpr int TPC = N * N / L;  // tiles per component
    __shared__ cx<T> lds[L * M];
    __shared__ cx<T> twl[N];
    for (int i = threadIdx.x; i < N; i += NT) twl[i] = pv.tw[i];
    cx<T> r0[NF], r1[NF];
    auto load = [&](int tile) {
        const int t = opaque((int)threadIdx.x);
        const int comp = tile / TPC;
        const cx<T>* in = comp == 0 ? in0 : (comp == 1 ? in1 : in2);
        const cx<T>* src = in + (uint64_t)(tile - comp * TPC) * L * M;
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const int fi = t + q * NT;
            r0[q] = src[2 * fi];
            r1[q] = src[2 * fi + 1];
        }
    };
    const uint64_t n3 = (uint64_t)N * N * N;
    // work-group b runs on XCD b % 8: with a grid of whole multiples of 8 each
    // XCD takes one contiguous eighth of the tiles (fewer pages in flight per
    // XCD), its work-groups striding through it
    int tile, tend, step;
    if ((gridDim.x & 7u) == 0) {
        const int per = (ntiles + 7) / 8;
        const int x = (int)(blockIdx.x & 7u);
        tile = x * per + (int)(blockIdx.x >> 3);
        tend = min(ntiles, (x + 1) * per);
        step = (int)(gridDim.x >> 3);
    } else {
        tile = blockIdx.x;
        tend = ntiles;
        step = (int)gridDim.x;
    }
    if (tile < tend) load(tile);
    for (; tile < tend; tile += step) {
        const int comp = tile / TPC;
        const uint64_t line0 = (uint64_t)(tile - comp * TPC) * L;
        // recomputed per tile rather than kept live across the loop
        const int t = opaque((int)threadIdx.x);
        const int c = t % L, j = t / L;
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const int fi = t + q * NT;
            const int cc = fi / (M / 2), k = 2 * (fi % (M / 2));
            cx<T> x0 = r0[q], x1 = r1[q];
            if (comp == 2) {
                x0 = cscale(x0, (T)k);
                x1 = cscale(x1, (T)(k + 1));
            }
            lds[lidx<L>(k, cc)] = x0;
            lds[lidx<L>(k + 1, cc)] = x1;
        }
        const int next = tile + step;
        load(next < tend ? next : tile);
        __syncthreads();
        cx<T> v[V];
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = c2r_pack<T, M, L>(lds, twl, (T)0, first_pos<M, 1>(j, i), c);
        __syncthreads();
        fft_lines<T, M, L, 1, 2>(v, lds, twl, c, j);
#pragma unroll
        for (int i = 0; i < V; ++i) lds[lidx<L>(last_pos<M, 1>(j, i), c)] = v[i];
        __syncthreads();
        // float tiles: a rolled loop keeps the kernel within 64 registers (two
        // work-groups per compute unit); double tiles are bound by LDS anyway
        constexpr int STORE_UNROLL = sizeof(T) == 8 ? NF : 1;
#pragma unroll STORE_UNROLL
        for (int q = 0; q < NF; ++q) {
            const int fi = t + q * NT;
            const int cc = fi / (M / 2), m = 2 * (fi % (M / 2));
            const cx<T> z0 = lds[lidx<L>(m, cc)], z1 = lds[lidx<L>(m + 1, cc)];
            int m0, m1;
            row_coords<true>(line0 + cc, N, m0, m1);
            const uint64_t off = (uint64_t)comp * n3 + ((uint64_t)m0 * N + m1) * N + 2 * m;
            if constexpr (PV) {
                const T vals[4] = {z0.x, z0.y, z1.x, z1.y};
                float p[4], u[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int mm = comp == 0 ? m0 : (comp == 1 ? m1 : 2 * m + e);
                    zel_point<T>(vals[e], mm, pv.origin[comp], pv.cell, pv.offset, pv.wrap, (T)pv.vfac, p[e], u[e]);
                }
                *reinterpret_cast<float4*>(za.pos + off) = make_float4(p[0], p[1], p[2], p[3]);
                *reinterpret_cast<float4*>(za.vel + off) = make_float4(u[0], u[1], u[2], u[3]);
            }
            if constexpr (PS) {
                T* o = static_cast<T*>(za.psi) + off;
                *reinterpret_cast<cx<T>*>(o) = z0;
                *reinterpret_cast<cx<T>*>(o + 2) = z1;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Strided passes: transforms of length N along an axis whose elements lie in
// separate rows, for L contiguous columns at a time (one 128-byte row chunk
// per element).  Tile blockIdx.x -> (outer index o, column block).  Element
// (o, p, col) is at obase(o) + poff(p) + col with
//   obase(o) = (o >> oshift) * ohi + (o & (2^oshift - 1)) * olo
//   poff(p)  = p * pstride,  or, with PBLK, (p >> 3) * phi + (p & 7) * plo.
// The blocked forms address the fused path's spectra, stored as
// [m0 / 8][k1][m0 % 8][k2] so that an axis-0 line touches N/8 far-apart
// regions of 8 neighbouring rows instead of N (fewer TLB misses).
//   SMODE_FWD / SMODE_INV : in0 -> out0 (may alias), forward / unnormalised inverse
//   SMODE_XFILT (P3)      : axis 0, o = k1: in0 -> F (out0), G (out1)
//   SMODE_YINV3 (P4)      : axis 1, o = m0: F (in0) -> A (out0), G (in1) -> B (out1), C (out2)
//   SMODE_YADJ (A2)       : axis 1, o = m0: forward transforms of two of the
//                           gradient's component spectra, Z = s1 FFT1(in0) + s2 FFT1(in1)
//                           -> out0 (the first, Y0, is a SMODE_FWD pass)
//   SMODE_XADJ (A3)       : adjoint of P3 + P4's axis-0 work: forward transforms of
//                           in0 (Y0) and in1 (Z), S = -i tau (s0 FFT0(Y0) + FFT0(Z))
//                           = -i tau (s0 X0 + s1 X1 + s2 X2), inverse -> out0
//   SMODE_XDELTA          : axis 0, o = k1: forward of in0, Eq. (1) factor
//                           sqrt(P N^3 / L^3) / N^3 = tau n^2 k_f, inverse -> out0
// A thread keeps one line's registers only: where a second transform of the
// same input is needed, the tile is read again (the re-read is served by the
// caches) rather than held, which keeps the kernels free of register spills.
// ---------------------------------------------------------------------------
enum {
    SMODE_FWD = 0,
    SMODE_INV = 1,
    SMODE_XFILT = 2,
    SMODE_YINV3 = 3,
    SMODE_XADJ = 4,
    SMODE_XDELTA = 5,
    SMODE_XWIN = 6,
    SMODE_YADJ = 7
};

template <typename T>
struct StridedArgs {
    const cx<T>* in0;
    const cx<T>* in1;
    const cx<T>* in2;
    cx<T>* out0;
    cx<T>* out1;
    cx<T>* out2;
    int64_t ohi, olo;
    int oshift;
    int64_t pstride;   // linear row stride (PBLK false)
    int64_t phi, plo;  // blocked row strides (PBLK true)
    int ncols;
    int ncb;  // column blocks per outer index in this launch
    int cb0;  // first column block of this launch
    int o0;   // first outer index of this launch
    int xgroup;  // tile order across XCDs (see xcd_tile)
    int64_t cstride;  // distance between the fields of blockIdx.y (0: one field)
};

// Tile of work-group b in a grid of nb work-groups.  The dispatcher hands
// work-group b to XCD b % 8; with xgroup = g > 0 each XCD takes groups of g
// consecutive tiles (g = 2: the two column blocks of neighbouring 128-byte
// chunks of the same rows), with g = 0 one contiguous range of nb / 8 tiles.
// A bijection on [0, nb): the last nb mod 8g work-groups keep their index.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb, int xgroup) {
    const unsigned g = xgroup > 0 ? (unsigned)xgroup : nb / 8u;
    if (g == 0) return b;
    const unsigned full = nb / (8u * g) * (8u * g);
    if (b >= full) return b;
    const unsigned x = b & 7u, k = b >> 3;
    return ((k / g) * 8u + x) * g + k % g;
}

template <typename T, int N, int MODE, int L, bool PBLK>
__global__ __launch_bounds__(L * PlanInfo<N>::TPL) void k_strided(StridedArgs<T> a, PlanView<T> pv) {
    constexpr int V = PlanInfo<N>::V;
    constexpr int TPL = PlanInfo<N>::TPL;
    static_assert(PlanInfo<N>::template last_radix<-1>() == PlanInfo<N>::template first_radix<1>(),
                  "inverse plan must start where the forward plan ends");
    __shared__ cx<T> lds[L * N];
    const int t = threadIdx.x;
    // y-passes (plain row strides) exchange the last stage across wave rows;
    // the x-passes keep the consecutive-row placement, whose four rows per
    // wave instruction sit in one blocked 8-row group
    constexpr bool RX = RowExchange<T, N, L>::value && !PBLK;
    const int c = t % L, j = line_thread<RX, L>(t);
    const unsigned tid = xcd_tile(blockIdx.x, gridDim.x, a.xgroup);
    const int o = a.o0 + (int)(tid / a.ncb);
    const int col0 = (a.cb0 + (int)(tid % a.ncb)) * L;
    const int col = col0 + c;
    const bool valid = col < a.ncols;
    // wave-uniform tile base; lanes past the last column of a ragged tile
    // re-read the last valid column (so every per-lane offset is >= 0) and
    // store nothing
    const int64_t tile = (int64_t)(o >> a.oshift) * a.ohi + (int64_t)(o & ((1 << a.oshift) - 1)) * a.olo + col0 +
                         (int64_t)blockIdx.y * a.cstride;
    const int cl = valid ? c : a.ncols - 1 - col0;
    auto poff = [&](int p) -> int64_t {
        if constexpr (PBLK) return (int64_t)(p >> 3) * a.phi + (int64_t)(p & 7) * a.plo;
        else return (int64_t)p * a.pstride;
    };
    // Slot i of a layout whose first (or only) stage has radix R sits at row
    // j + TPL (i / R) + (i % R) N / R.  When the compile-time row part is a
    // multiple of 8 the address splits into a wave-uniform slot pointer
    // (scalar registers) plus one 32-bit per-lane byte offset.
    constexpr bool SPLIT = (TPL % 8 == 0) && (N % 128 == 0);
    auto lane_bytes = [&](int jj) -> uint32_t {
        return SPLIT ? (uint32_t)((poff(jj) + cl) * (int64_t)sizeof(cx<T>)) : 0u;
    };
    auto at = [&](auto* base, int i, int R, int jj, uint32_t laneb) {
        const int rowc = TPL * (i / R) + (i % R) * (N / R);
        using P = decltype(base);
        if constexpr (SPLIT) {
            auto* slot = base + (tile + poff(rowc));
            using B = std::conditional_t<std::is_const_v<std::remove_pointer_t<P>>, const char*, char*>;
            return reinterpret_cast<P>(reinterpret_cast<B>(slot) + laneb);
        } else {
            return base + (tile + cl + poff(jj + rowc));
        }
    };
    constexpr int RF = PlanInfo<N>::template first_radix<-1>();  // forward input layout
    constexpr int RL = PlanInfo<N>::template last_radix<1>();    // inverse output layout
    constexpr int RM = PlanInfo<N>::template last_radix<-1>();   // forward output = inverse input
    cx<T> v[V];

    if constexpr (MODE == SMODE_FWD || MODE == SMODE_INV) {
        constexpr int DIR = MODE == SMODE_FWD ? -1 : 1;
        constexpr int RI = DIR < 0 ? RF : RM;
        constexpr int RO = DIR < 0 ? RM : RL;
        const uint32_t lb = lane_bytes(j);
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = *at(a.in0, i, RI, j, lb);
        fft_lines<T, N, L, DIR, 1, RX>(v, lds, pv.tw, c, j);
        if (valid) {
#pragma unroll
            for (int i = 0; i < V; ++i) *at(a.out0, i, RO, j, lb) = v[i];
        }
    } else if constexpr (MODE == SMODE_XFILT) {
        const TauLookup<T> taul = tau_lookup(pv);
        const uint32_t lb = lane_bytes(j);
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = *at(a.in0, i, RF, j, lb);
        __syncthreads();
        fft_lines<T, N, L, -1, 1, RX>(v, lds, pv.tw, c, j);
        // Eq. (1)-(2) on the spectrum held in registers (positions = axis-0 modes)
        const int s1 = signed_mode(o, N);
        const int s2 = col;
        const bool line_zero = (s1 == -(N / 2)) || (s2 >= N / 2);
        const T dline = pv.deconv ? cic_deconv<T>(s1, N) * cic_deconv<T>(s2, N) : (T)1;
        cx<T> g[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int k0 = last_pos<N, -1>(j, i);
            const int s0 = signed_mode(k0, N);
            const int n2 = s0 * s0 + s1 * s1 + s2 * s2;
            const bool zero = line_zero || (k0 == N / 2) || n2 < pv.n2_lo || n2 >= pv.n2_hi;
            T tau = taul(zero ? 0 : n2) * (T)pv.amp_scale;  // tau(0) = 0: mean and Nyquist vanish
            if (pv.deconv) tau *= cic_deconv<T>(s0, N) * dline;
            g[i] = mul_i(cscale(v[i], tau));
            v[i] = cscale(g[i], (T)s0);
        }
        {
            const int jj = opaque(j), cc = opaque(c);
            fft_lines<T, N, L, 1, 1, RX>(v, lds, pv.tw, cc, jj);
            const uint32_t lb2 = lane_bytes(jj);
            if (valid) {
#pragma unroll
                for (int i = 0; i < V; ++i) *at(a.out0, i, RL, jj, lb2) = v[i];
            }
        }
        {
            const int jj = opaque(j), cc = opaque(c);
            fft_lines<T, N, L, 1, 1, RX>(g, lds, pv.tw, cc, jj);
            const uint32_t lb2 = lane_bytes(jj);
            if (valid) {
#pragma unroll
                for (int i = 0; i < V; ++i) *at(a.out1, i, RL, jj, lb2) = g[i];
            }
        }
    } else if constexpr (MODE == SMODE_YADJ) {
        // Z = s1 FFT1(in0) + s2 FFT1(in1) -> out0.  At N = 1024, while the second
        // line is transformed, PK of the first line's values wait in the LDS
        // left over beside the tile (its registers would spill otherwise; smaller
        // plans fit, and extra LDS would cost them work-groups per CU)
        constexpr int NT = L * TPL;
        constexpr int FREE = (160 * 1024 - (int)sizeof(cx<T>) * L * N) / ((int)sizeof(cx<T>) * NT);
        constexpr int PK = N < 1024 ? 0 : (FREE < V ? FREE : V);
        __shared__ cx<T> park[(PK > 0 ? PK : 1) * NT];
        cx<T> g[V];
        {
            const uint32_t lb = lane_bytes(j);
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = *at(a.in0, i, RF, j, lb);
            fft_lines<T, N, L, -1, 1, RX>(v, lds, pv.tw, c, j);
            const int jk = opaque(j);
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = cscale(v[i], (T)signed_mode(last_pos<N, -1>(jk, i), N));
            const int tt = opaque((int)threadIdx.x);
#pragma unroll
            for (int i = 0; i < PK; ++i) park[i * NT + tt] = v[V - PK + i];
        }
        {
            const int jj = opaque(j), cc = opaque(c);
            const uint32_t lb = lane_bytes(jj);
#pragma unroll
            for (int i = 0; i < V; ++i) g[i] = *at(a.in1, i, RF, jj, lb);
            fft_lines<T, N, L, -1, 1, RX>(g, lds, pv.tw, cc, jj);
            const int tt = opaque((int)threadIdx.x);
#pragma unroll
            for (int i = 0; i < PK; ++i) v[V - PK + i] = park[i * NT + tt];
            const T s2 = (T)col;
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = cadd(v[i], cscale(g[i], s2));
            const uint32_t lb2 = lane_bytes(jj);
            if (valid) {
#pragma unroll
                for (int i = 0; i < V; ++i) *at(a.out0, i, RM, jj, lb2) = v[i];
            }
        }
    } else if constexpr (MODE == SMODE_XADJ) {
        const TauLookup<T> taul = tau_lookup(pv);
        __syncthreads();
        const int s1 = signed_mode(o, N);
        const int s2 = col;
        const bool line_zero = (s1 == -(N / 2)) || (s2 >= N / 2);
        // A2 has already formed Z = s1 Y1 + s2 Y2 (s1 and s2 are constant along
        // an axis-0 line): two forward transforms, Z and Y0 loaded together
        cx<T> acc[V];
        {
            const uint32_t lb = lane_bytes(j);
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = *at(a.in1, i, RF, j, lb);
#pragma unroll
            for (int i = 0; i < V; ++i) acc[i] = *at(a.in0, i, RF, j, lb);
        }
        {
            const int jj = opaque(j), cc = opaque(c);
            fft_lines<T, N, L, -1, 1, RX>(v, lds, pv.tw, cc, jj);
        }
        {
            const int jj = opaque(j), cc = opaque(c);
            fft_lines<T, N, L, -1, 1, RX>(acc, lds, pv.tw, cc, jj);
            const int jk = opaque(jj);
#pragma unroll
            for (int i = 0; i < V; ++i)
                acc[i] = cadd(cscale(acc[i], (T)signed_mode(last_pos<N, -1>(jk, i), N)), v[i]);
        }
        {
            const int jj = opaque(j), cc = opaque(c);
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const int k0 = last_pos<N, -1>(jj, i);
                const int s0 = signed_mode(k0, N);
                const int n2 = s0 * s0 + s1 * s1 + s2 * s2;
                const bool zero = line_zero || (k0 == N / 2);
                const T tau = taul(zero ? 0 : n2) * (T)pv.amp_scale;
                v[i] = mul_i(cscale(acc[i], -tau));
            }
            fft_lines<T, N, L, 1, 1, RX>(v, lds, pv.tw, cc, jj);
            const uint32_t lb = lane_bytes(jj);
            if (valid) {
#pragma unroll
                for (int i = 0; i < V; ++i) *at(a.out0, i, RL, jj, lb) = v[i];
            }
        }
    } else if constexpr (MODE == SMODE_XWIN) {
        // axis-0 forward, the Eq. 5 window n2_lo <= n^2 < n2_hi (with the
        // cloud-in-cell deconvolution if set), axis-0 inverse; in0 -> out0
        const uint32_t lb = lane_bytes(j);
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = *at(a.in0, i, RF, j, lb);
        __syncthreads();
        fft_lines<T, N, L, -1, 1, RX>(v, lds, pv.tw, c, j);
        const int s1 = signed_mode(o, N);
        const int s2 = col;
        const bool line_zero = (s1 == -(N / 2)) || (s2 >= N / 2);
        const T dline = pv.deconv ? cic_deconv<T>(s1, N) * cic_deconv<T>(s2, N) : (T)1;
        const int jj = opaque(j);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int k0 = last_pos<N, -1>(jj, i);
            const int s0 = signed_mode(k0, N);
            const int n2 = s0 * s0 + s1 * s1 + s2 * s2;
            const bool zero = line_zero || (k0 == N / 2) || n2 < pv.n2_lo || n2 >= pv.n2_hi;
            T f = zero ? (T)0 : (T)1;
            if (pv.deconv) f *= cic_deconv<T>(s0, N) * dline;
            v[i] = cscale(v[i], f);
        }
        const int cc = opaque(c);
        fft_lines<T, N, L, 1, 1, RX>(v, lds, pv.tw, cc, jj);
        const uint32_t lb2 = lane_bytes(jj);
        if (valid) {
#pragma unroll
            for (int i = 0; i < V; ++i) *at(a.out0, i, RL, jj, lb2) = v[i];
        }
    } else if constexpr (MODE == SMODE_XDELTA) {
        const TauLookup<T> taul = tau_lookup(pv);
        const uint32_t lb = lane_bytes(j);
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = *at(a.in0, i, RF, j, lb);
        __syncthreads();
        fft_lines<T, N, L, -1, 1, RX>(v, lds, pv.tw, c, j);
        const int s1 = signed_mode(o, N);
        const int s2 = col;
        const bool line_zero = (s1 == -(N / 2)) || (s2 >= N / 2);
        const T kf = (T)(2.0 * 3.14159265358979323846 / pv.box);
        const T dline = pv.deconv ? cic_deconv<T>(s1, N) * cic_deconv<T>(s2, N) : (T)1;
        const int jj = opaque(j), cc = opaque(c);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int k0 = last_pos<N, -1>(jj, i);
            const int s0 = signed_mode(k0, N);
            const int n2 = s0 * s0 + s1 * s1 + s2 * s2;
            const bool zero = line_zero || (k0 == N / 2) || n2 < pv.n2_lo || n2 >= pv.n2_hi;
            T f = taul(zero ? 0 : n2) * ((T)n2 * kf);
            if (pv.deconv) f *= cic_deconv<T>(s0, N) * dline;
            v[i] = cscale(v[i], f);
        }
        fft_lines<T, N, L, 1, 1, RX>(v, lds, pv.tw, cc, jj);
        const uint32_t lb2 = lane_bytes(jj);
        if (valid) {
#pragma unroll
            for (int i = 0; i < V; ++i) *at(a.out0, i, RL, jj, lb2) = v[i];
        }
    } else {  // SMODE_YINV3
        // float tiles load G together with F: its reads are in flight during
        // A's transform and stores (one work-group per compute unit, so nothing
        // else would hide them); double tiles (two work-groups' worth of
        // registers already) measured faster loading G after A
        constexpr bool EARLY_G = sizeof(T) == 4;
        cx<T> g[V];
        {
            const uint32_t lb = lane_bytes(j);
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = *at(a.in0, i, RM, j, lb);
            if constexpr (EARLY_G) {
#pragma unroll
                for (int i = 0; i < V; ++i) g[i] = *at(a.in1, i, RM, j, lb);
            }
            fft_lines<T, N, L, 1, 1, RX>(v, lds, pv.tw, c, j);
            if (valid) {
#pragma unroll
                for (int i = 0; i < V; ++i) *at(a.out0, i, RL, j, lb) = v[i];
            }
        }
        {
            const int jj = opaque(j), cc = opaque(c);
            const uint32_t lb = lane_bytes(jj);
            if constexpr (!EARLY_G) {
#pragma unroll
                for (int i = 0; i < V; ++i) g[i] = *at(a.in1, i, RM, jj, lb);
            }
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = cscale(g[i], (T)signed_mode(first_pos<N, 1>(jj, i), N));
            fft_lines<T, N, L, 1, 1, RX>(v, lds, pv.tw, cc, jj);
            if (valid) {
#pragma unroll
                for (int i = 0; i < V; ++i) *at(a.out1, i, RL, jj, lb) = v[i];
            }
        }
        {
            const int jj = opaque(j), cc = opaque(c);
            const uint32_t lb = lane_bytes(jj);
            fft_lines<T, N, L, 1, 1, RX>(g, lds, pv.tw, cc, jj);
            if (valid) {
#pragma unroll
                for (int i = 0; i < V; ++i) *at(a.out2, i, RL, jj, lb) = g[i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// P3 for float plans as a persistent kernel (same arithmetic as SMODE_XFILT
// above).  Work-group b takes tiles b, b + G, ... (G = gridDim.x, tile order
// across XCDs by xcd_tile over the launch's ntiles tiles).  Once F is
// stored, the registers of its line are free: the next tile's input is
// loaded into them and is in flight while G is transformed and stored.  The
// twiddles are copied into LDS once, so that no global load follows the
// prefetch (loads complete in order).  LDS: tile 128 KB + twiddles 8 KB +
// tau segments 15 KB at N = 1024, one work-group per compute unit.
// ---------------------------------------------------------------------------
template <typename T, int N, int L>
__global__ __launch_bounds__(L * PlanInfo<N>::TPL) void k_xfilt(StridedArgs<T> a, PlanView<T> pv, int ntiles) {
    static_assert(std::is_same_v<T, float>, "double tiles leave no LDS for the twiddle table");
    constexpr int V = PlanInfo<N>::V;
    constexpr int TPL = PlanInfo<N>::TPL;
    constexpr int RF = PlanInfo<N>::template first_radix<-1>();
    constexpr int RL = PlanInfo<N>::template last_radix<1>();
    constexpr bool SPLIT = (TPL % 8 == 0) && (N % 128 == 0);
    __shared__ cx<T> lds[L * N];
    __shared__ cx<T> twl[N];
    for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = pv.tw[i];
    const TauLookup<T> taul = tau_lookup(pv);
    auto poff = [&](int p) -> int64_t { return (int64_t)(p >> 3) * a.phi + (int64_t)(p & 7) * a.plo; };
    struct TileAt {
        int o, col, cl;
        bool valid;
        int64_t base;  // wave-uniform
    };
    auto tile_at = [&](int u, int c) -> TileAt {
        const unsigned tid = xcd_tile((unsigned)u, (unsigned)ntiles, a.xgroup);
        TileAt r;
        r.o = a.o0 + (int)(tid / a.ncb);
        const int col0 = (a.cb0 + (int)(tid % a.ncb)) * L;
        r.col = col0 + c;
        r.valid = r.col < a.ncols;
        r.cl = r.valid ? c : a.ncols - 1 - col0;
        r.base = (int64_t)(r.o >> a.oshift) * a.ohi + (int64_t)(r.o & ((1 << a.oshift) - 1)) * a.olo + col0;
        return r;
    };
    // slot i of line thread jj (layout radix R), as in k_strided
    auto at = [&](auto* base, const TileAt& tl, int i, int R, int jj) {
        const int rowc = TPL * (i / R) + (i % R) * (N / R);
        using P = decltype(base);
        if constexpr (SPLIT) {
            auto* slot = base + (tl.base + poff(rowc));
            using B = std::conditional_t<std::is_const_v<std::remove_pointer_t<P>>, const char*, char*>;
            const uint32_t laneb = (uint32_t)((poff(jj) + tl.cl) * (int64_t)sizeof(cx<T>));
            return reinterpret_cast<P>(reinterpret_cast<B>(slot) + laneb);
        } else {
            return base + (tl.base + tl.cl + poff(jj + rowc));
        }
    };
    cx<T> v[V];
    int u = blockIdx.x;
    {
        const int t = opaque((int)threadIdx.x);
        const TileAt tl = tile_at(u < ntiles ? u : 0, t % L);
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = *at(a.in0, tl, i, RF, t / L);
    }
    __syncthreads();
    for (; u < ntiles; u += gridDim.x) {
        const int t = opaque((int)threadIdx.x);
        const int c = t % L, j = t / L;
        const TileAt tl = tile_at(u, c);
        fft_lines<T, N, L, -1, 1>(v, lds, twl, c, j);
        const int s1 = signed_mode(tl.o, N);
        const int s2 = tl.col;
        const bool line_zero = (s1 == -(N / 2)) || (s2 >= N / 2);
        const T dline = pv.deconv ? cic_deconv<T>(s1, N) * cic_deconv<T>(s2, N) : (T)1;
        cx<T> g[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int k0 = last_pos<N, -1>(j, i);
            const int s0 = signed_mode(k0, N);
            const int n2 = s0 * s0 + s1 * s1 + s2 * s2;
            const bool zero = line_zero || (k0 == N / 2) || n2 < pv.n2_lo || n2 >= pv.n2_hi;
            T tau = taul(zero ? 0 : n2) * (T)pv.amp_scale;  // tau(0) = 0: mean and Nyquist vanish
            if (pv.deconv) tau *= cic_deconv<T>(s0, N) * dline;
            g[i] = mul_i(cscale(v[i], tau));
            v[i] = cscale(g[i], (T)s0);
        }
        {
            const int jj = opaque(j), cc = opaque(c);
            fft_lines<T, N, L, 1, 1>(v, lds, twl, cc, jj);
            const TileAt to = tile_at(opaque(u), cc);
            if (to.valid) {
#pragma unroll
                for (int i = 0; i < V; ++i) *at(a.out0, to, i, RL, jj) = v[i];
            }
        }
        {
            // the next tile (this one again after the last) into v
            const int jj = opaque(j), cc = opaque(c);
            const int un = u + (int)gridDim.x;
            const TileAt tn = tile_at(un < ntiles ? un : u, cc);
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = *at(a.in0, tn, i, RF, jj);
        }
        {
            const int jj = opaque(j), cc = opaque(c);
            fft_lines<T, N, L, 1, 1>(g, lds, twl, cc, jj);
            const TileAt to = tile_at(opaque(u), cc);
            if (to.valid) {
#pragma unroll
                for (int i = 0; i < V; ++i) *at(a.out1, to, i, RL, jj) = g[i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Eq. 5 window on a plain half spectrum (rows (k0, k1), k2 in [0, N/2]):
// modes with n^2 >= n2_max are zeroed, the others divided by the CiC window
// prod_j sinc^2(pi s_j / N) if deconv is set.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_window(cx<T>* __restrict__ spec, int n, int n2_max, int deconv) {
    const uint32_t K = n / 2 + 1;
    const uint32_t total = (uint32_t)n * n * K;  // < 2^30 for n <= 1024
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int k2 = (int)(i % K);
        const uint32_t r = i / K;
        const int k1 = (int)(r % (uint32_t)n), k0 = (int)(r / (uint32_t)n);
        const int s0 = k0 <= n / 2 ? k0 : k0 - n, s1 = k1 <= n / 2 ? k1 : k1 - n;
        const int n2 = s0 * s0 + s1 * s1 + k2 * k2;
        T f = n2 < n2_max ? (T)1 : (T)0;
        if (deconv && n2 < n2_max) f = cic_deconv<T>(s0, n) * cic_deconv<T>(s1, n) * cic_deconv<T>(k2, n);
        spec[i] = cscale(spec[i], f);
    }
}

// ---------------------------------------------------------------------------
// Resolution degrade (Sec. 2.3): nearest-grid-point values of a periodic
// fine field on the coarse lattice, whose point m coincides with fine point
// factor * m ...
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_decimate(const T* __restrict__ fine, int n_lo, int factor, T* __restrict__ lo) {
    const uint64_t total = (uint64_t)n_lo * n_lo * n_lo;
    const uint64_t n_hi = (uint64_t)n_lo * factor;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t m2 = i % n_lo, r = i / n_lo;
        const uint64_t m1 = r % n_lo, m0 = r / n_lo;
        lo[i] = fine[((m0 * factor) * n_hi + m1 * factor) * n_hi + m2 * factor];
    }
}

// ... then moved by s_j coarse cells along axis j in Fourier space: mode n
// (signed) gets exp(-2 pi i s n / N) per axis, the Nyquist plane cos(pi s)
// (the real band-limited interpolant), on a plain half spectrum.
template <typename T>
__device__ __forceinline__ cx<T> translate_factor(int k, int n, double s) {
    if (2 * k == n) return {(T)cospi(s), (T)0};
    const int sk = k <= n / 2 ? k : k - n;
    double a = -2.0 * s * (double)sk / (double)n;  // angle in units of pi
    a -= 2.0 * rint(0.5 * a);                      // into [-1, 1]
    T sn, cs;
    if constexpr (sizeof(T) == 4) sincospif((float)a, &sn, &cs);
    else sincospi(a, &sn, &cs);
    return {cs, sn};
}

template <typename T>
__global__ void k_translate(cx<T>* __restrict__ spec, int n, double s0, double s1, double s2) {
    const uint32_t K = n / 2 + 1;
    const uint32_t total = (uint32_t)n * n * K;  // < 2^30 for n <= 1024
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int k2 = (int)(i % K);
        const uint32_t r = i / K;
        const int k1 = (int)(r % (uint32_t)n), k0 = (int)(r / (uint32_t)n);
        const cx<T> f = cmul(cmul(translate_factor<T>(k0, n, s0), translate_factor<T>(k1, n, s1)),
                             translate_factor<T>(k2, n, s2));
        spec[i] = cmul(spec[i], f);
    }
}

// ---------------------------------------------------------------------------
// Stand-alone Eq. (1)-(2) on a full half spectrum (k2 in [0, N/2]).
// tau here carries the 1/N^3 of the fused path; scale = N^3 removes it.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_filter(const cx<T>* __restrict__ w, cx<T>* __restrict__ psi, cx<T>* __restrict__ delta, int n,
                         T scale, T kf, PlanView<T> pv) {
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
        const T ts = pv.tau[zero ? 0 : n2] * scale;
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
    // block: one lattice row (m0, m1) = blockIdx.x and a run of m2; comp = blockIdx.z
    const int n = pv.n;
    const int m2 = blockIdx.y * blockDim.x + threadIdx.x;
    if (m2 >= n) return;
    const int row = blockIdx.x;
    const int m0 = row / n, m1 = row - m0 * n;
    const int comp = blockIdx.z;
    const uint64_t idx = (uint64_t)comp * n * n * n + (uint64_t)row * n + m2;
    const int m = comp == 0 ? m0 : (comp == 1 ? m1 : m2);
    zel_point<T>(psi[idx], m, pv.origin[comp], pv.cell, pv.offset, pv.wrap, (T)pv.vfac, pos[idx], vel[idx]);
}

}  // namespace gg
