// White-noise refinement (App. A) and cloud-in-cell interpolation of a coarse
// field onto a finer lattice of the same box (Sec. 2.3, Eq. 4-5).
//
// Refinement: a patch of NL^3 parent cells becomes NH^3 child cells.  With
// orthonormal 1D bases F_i (NL points, Eq. A.5-A.6, or F_0 = [1] for NL = 1)
// and E_j (NH points), the parent coefficients a_ijk = sum V F_i F_j F_k
// (i, j, k < NL) are kept, every coefficient with an index >= NL is a new
// unit Gaussian, and the child patch is sum a_ijk E_i E_j E_k (Eq. A.28).
// The new coefficient (i, j, k) of patch p (row-major over the patch grid) is
// the binary64 noise value of index p NH^3 + (i NH + j) NH + k for the given
// seed and stream (one Philox call, as one noise cell).  One thread refines
// one patch in binary64; the child values are rounded once to T.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "noise_dev.h"

namespace gg {

// basis variants (the C ABI's gg_refine values)
enum { REFINE_HR = 0, REFINE_3 = 1, REFINE_4 = 2, REFINE_LINEAR = 3, REFINE_SINE = 4 };

template <int V>
struct RefineBasis;

template <>
struct RefineBasis<REFINE_HR> {
    static constexpr int NL = 1, NH = 2;
    __device__ static double E(int j, int m) {
        const double h = 0.70710678118654752440;  // 1/sqrt(2)
        return j == 0 ? h : (m == 0 ? -h : h);
    }
};

template <>
struct RefineBasis<REFINE_3> {
    static constexpr int NL = 2, NH = 3;
    __device__ static double E(int j, int m) {
        const double r3 = 0.57735026918962576451, r2 = 0.70710678118654752440, r6 = 0.40824829046386301637;
        if (j == 0) return r3;
        if (j == 1) return m == 0 ? -r2 : (m == 1 ? 0.0 : r2);
        return m == 1 ? 2.0 * r6 : -r6;
    }
};

template <>
struct RefineBasis<REFINE_4> {
    static constexpr int NL = 2, NH = 4;
    __device__ static double E(int j, int m) {
        const double q7 = 0.66143782776614764763;  // sqrt(7)/4
        const double e1[4] = {-q7, -0.25, 0.25, q7};
        const double e2[4] = {-0.5, 0.5, 0.5, -0.5};
        const double e3[4] = {0.25, -q7, q7, -0.25};
        return j == 0 ? 0.5 : (j == 1 ? e1[m] : (j == 2 ? e2[m] : e3[m]));
    }
};

template <>
struct RefineBasis<REFINE_LINEAR> {
    static constexpr int NL = 2, NH = 4;
    __device__ static double E(int j, int m) {
        const double r = 0.22360679774997896964;  // 1/sqrt(20)
        const double e1[4] = {-3.0 * r, -r, r, 3.0 * r};
        const double e2[4] = {-0.5, 0.5, 0.5, -0.5};
        const double e3[4] = {r, -3.0 * r, 3.0 * r, -r};
        return j == 0 ? 0.5 : (j == 1 ? e1[m] : (j == 2 ? e2[m] : e3[m]));
    }
};

template <>
struct RefineBasis<REFINE_SINE> {
    static constexpr int NL = 2, NH = 4;
    __device__ static double E(int j, int m) {
        const double e1[4] = {-0.5, -0.5, 0.5, 0.5};
        const double e2[4] = {-0.5, 0.5, 0.5, -0.5};
        const double e3[4] = {0.5, -0.5, 0.5, -0.5};
        return j == 0 ? 0.5 : (j == 1 ? e1[m] : (j == 2 ? e2[m] : e3[m]));
    }
};

// parent basis F (Eq. A.5-A.6 for NL = 2)
template <int NL>
__device__ inline double refine_F(int i, int m) {
    if constexpr (NL == 1) {
        return 1.0;
    } else {
        const double h = 0.70710678118654752440;
        return i == 0 ? h : (m == 0 ? -h : h);
    }
}

// One thread per patch, 64 patches (one wave) per work-group; P patches per
// axis over the parent cells o + [0, P NL) (periodic in the npar^3 parent);
// child (P NH)^3.  The NH^3 coefficients of each patch
// sit in LDS ([coefficient][thread], conflict-free); the three 1D expansions
// run in place there.
constexpr int kRefineThreads = 64;

template <typename T, int VAR>
__global__ __launch_bounds__(kRefineThreads) void k_refine(const T* __restrict__ parent, int npar, int o0, int o1,
                                                           int o2, int P, uint64_t seed, uint32_t stream,
                                                           T* __restrict__ child) {
    using B = RefineBasis<VAR>;
    constexpr int NL = B::NL, NH = B::NH, NC = NH * NH * NH;
    __shared__ double coef[NC * kRefineThreads];
    const int t = threadIdx.x;
    auto A = [&](int i, int j, int k) -> double& { return coef[((i * NH + j) * NH + k) * kRefineThreads + t]; };
    const uint64_t np = (uint64_t)P * P * P;
    const uint64_t p = (uint64_t)blockIdx.x * kRefineThreads + t;
    if (p >= np) return;  // no barriers below: each thread works on its own LDS column
    const int p2 = (int)(p % P), p1 = (int)((p / P) % P), p0 = (int)(p / ((uint64_t)P * P));
    const int64_t nch = (int64_t)P * NH;
    // new coefficients: every index combination with an index >= NL
#pragma unroll 1
    for (int q = 0; q < NC; ++q) {
        const int i = q / (NH * NH), j = (q / NH) % NH, k = q % NH;
        if (i >= NL || j >= NL || k >= NL) coef[q * kRefineThreads + t] = gaussian_cell(p * (uint64_t)NC + q, seed, stream);
    }
    // parent coefficients a_ijk = sum_mnl V(m, n, l) F_i(m) F_j(n) F_k(l)
    double v[NL][NL][NL];
#pragma unroll
    for (int m = 0; m < NL; ++m)
#pragma unroll
        for (int n = 0; n < NL; ++n)
#pragma unroll
            for (int l = 0; l < NL; ++l)
                v[m][n][l] = (double)parent[((int64_t)((o0 + p0 * NL + m) % npar) * npar + (o1 + p1 * NL + n) % npar) * npar +
                                            (o2 + p2 * NL + l) % npar];
#pragma unroll
    for (int i = 0; i < NL; ++i)
#pragma unroll
        for (int j = 0; j < NL; ++j)
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                double s = 0.0;
#pragma unroll
                for (int m = 0; m < NL; ++m)
#pragma unroll
                    for (int n = 0; n < NL; ++n)
#pragma unroll
                        for (int l = 0; l < NL; ++l)
                            s += v[m][n][l] * refine_F<NL>(i, m) * refine_F<NL>(j, n) * refine_F<NL>(k, l);
                A(i, j, k) = s;
            }
    // expand along axis 2, then 1, then 0 (in place, one line of NH at a time)
#pragma unroll
    for (int i = 0; i < NH; ++i)
#pragma unroll
        for (int j = 0; j < NH; ++j) {
            double x[NH], y[NH];
#pragma unroll
            for (int k = 0; k < NH; ++k) x[k] = A(i, j, k);
#pragma unroll
            for (int l = 0; l < NH; ++l) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < NH; ++k) s += x[k] * B::E(k, l);
                y[l] = s;
            }
#pragma unroll
            for (int l = 0; l < NH; ++l) A(i, j, l) = y[l];
        }
#pragma unroll
    for (int i = 0; i < NH; ++i)
#pragma unroll
        for (int l = 0; l < NH; ++l) {
            double x[NH], y[NH];
#pragma unroll
            for (int j = 0; j < NH; ++j) x[j] = A(i, j, l);
#pragma unroll
            for (int n = 0; n < NH; ++n) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < NH; ++j) s += x[j] * B::E(j, n);
                y[n] = s;
            }
#pragma unroll
            for (int n = 0; n < NH; ++n) A(i, n, l) = y[n];
        }
#pragma unroll
    for (int n = 0; n < NH; ++n)
#pragma unroll
        for (int l = 0; l < NH; ++l) {
            double x[NH], y[NH];
#pragma unroll
            for (int i = 0; i < NH; ++i) x[i] = A(i, n, l);
#pragma unroll
            for (int m = 0; m < NH; ++m) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < NH; ++i) s += x[i] * B::E(i, m);
                y[m] = s;
            }
#pragma unroll
            for (int m = 0; m < NH; ++m) A(m, n, l) = y[m];
        }
#pragma unroll
    for (int m = 0; m < NH; ++m)
#pragma unroll
        for (int n = 0; n < NH; ++n) {
            T* row = child + (((int64_t)p0 * NH + m) * nch + (int64_t)p1 * NH + n) * nch + (int64_t)p2 * NH;
#pragma unroll
            for (int l = 0; l < NH; ++l) row[l] = (T)A(m, n, l);
        }
}

// dst (3 fields of nd^3) += trilinear interpolation of the periodic src (3
// fields of ns^3) at the points u = o + m num / den (src cells), m < nd per
// axis (num / den = 1 / R for a refinement by an integer R, n_src / n_dst in
// lowest terms for a whole box resampled to another size).  Cell and weight
// come from exact integer arithmetic; products and sums in binary64, then
// rounded to T.  A work-group covers one destination row (x, y) and a run of
// z: the row's cells and weights along axes 0 and 1 are the same for every
// thread, and each thread does all three fields, so the integer arithmetic
// is done once per point and 24 independent loads are in flight per thread.
// ZEL: the point's final displacement also gives its particle (Eq. 3 on the
// lattice of pv, as k_zeldovich): a zoom level's particles without reading
// the field back.
template <typename T, bool ZEL>
__global__ void k_cic_add(const T* __restrict__ src, int ns, int num, int den, int o0, int o1, int o2,
                          T* __restrict__ dst, int nd, PlanView<T> pv, float* __restrict__ pos,
                          float* __restrict__ vel) {
    const int z = blockIdx.y * blockDim.x + threadIdx.x;
    if (z >= nd) return;
    const int row = blockIdx.x;
    const int x = row / nd, y = row - x * nd;
    const uint64_t n3d = (uint64_t)nd * nd * nd;
    const uint64_t n3s = (uint64_t)ns * ns * ns;
    // point m sits at o + m num / den source cells: cell o + floor(m num / den), weight (m num mod den) / den
    const int xn = x * num, yn = y * num, zn = z * num;
    const int x0 = (o0 + xn / den) % ns, y0 = (o1 + yn / den) % ns, z0 = (o2 + zn / den) % ns;
    const double tx = (double)(xn % den) / den, ty = (double)(yn % den) / den, tz = (double)(zn % den) / den;
    const int x1 = x0 + 1 == ns ? 0 : x0 + 1, y1 = y0 + 1 == ns ? 0 : y0 + 1, z1 = z0 + 1 == ns ? 0 : z0 + 1;
    // offsets of the four (axis 0, axis 1) corners' rows
    const uint64_t r00 = ((uint64_t)x0 * ns + y0) * ns, r10 = ((uint64_t)x1 * ns + y0) * ns;
    const uint64_t r01 = ((uint64_t)x0 * ns + y1) * ns, r11 = ((uint64_t)x1 * ns + y1) * ns;
    T c[3][8];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        const T* s = src + comp * n3s;
        c[comp][0] = s[r00 + z0];
        c[comp][1] = s[r10 + z0];
        c[comp][2] = s[r01 + z0];
        c[comp][3] = s[r11 + z0];
        c[comp][4] = s[r00 + z1];
        c[comp][5] = s[r10 + z1];
        c[comp][6] = s[r01 + z1];
        c[comp][7] = s[r11 + z1];
    }
    T* d = dst + (uint64_t)row * nd + z;
    T old[3];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) old[comp] = d[comp * n3d];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        // interpolate along axis 0, then 1, then 2 (the oracle's order)
        const double a00 = (double)c[comp][0] * (1.0 - tx) + (double)c[comp][1] * tx;
        const double a10 = (double)c[comp][2] * (1.0 - tx) + (double)c[comp][3] * tx;
        const double a01 = (double)c[comp][4] * (1.0 - tx) + (double)c[comp][5] * tx;
        const double a11 = (double)c[comp][6] * (1.0 - tx) + (double)c[comp][7] * tx;
        const double b0 = a00 * (1.0 - ty) + a10 * ty;
        const double b1 = a01 * (1.0 - ty) + a11 * ty;
        const double v = b0 * (1.0 - tz) + b1 * tz;
        const T out = (T)((double)old[comp] + v);
        d[comp * n3d] = out;
        if constexpr (ZEL) {
            const uint64_t idx = comp * n3d + (uint64_t)row * nd + z;
            zel_point<T>(out, comp == 0 ? x : (comp == 1 ? y : z), pv.origin[comp], pv.cell, pv.offset, pv.wrap,
                         (T)pv.vfac, pos[idx], vel[idx]);
        }
    }
}

}  // namespace gg
