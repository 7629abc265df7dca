// Definitions of Ops<T>: grid shapes and the pass sequence of the fused path.
#pragma once
#include <type_traits>

#include "cosmo_dev.h"
#include "kernels.h"
#include "ops.h"

namespace gg {

template <typename F>
hipError_t dispatch_n(int n, F&& f) {
    switch (n) {
        case 8: return f(std::integral_constant<int, 8>{});
        case 16: return f(std::integral_constant<int, 16>{});
        case 32: return f(std::integral_constant<int, 32>{});
        case 64: return f(std::integral_constant<int, 64>{});
        case 128: return f(std::integral_constant<int, 128>{});
        case 256: return f(std::integral_constant<int, 256>{});
        case 512: return f(std::integral_constant<int, 512>{});
        case 1024: return f(std::integral_constant<int, 1024>{});
        default: return hipErrorInvalidValue;
    }
}

inline unsigned capped_grid(uint64_t work, unsigned block) {
    uint64_t g = (work + block - 1) / block;
    const uint64_t cap = 256ull * 64ull;
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

template <typename T>
StridedArgs<T> strided_args(const cx<T>* in0, const cx<T>* in1, cx<T>* out0, cx<T>* out1, cx<T>* out2, int64_t ohi,
                            int64_t olo, int oshift, int64_t pstride, int64_t phi, int64_t plo, int ncols) {
    return StridedArgs<T>{in0, in1, out0, out1, out2, ohi, olo, oshift, pstride, phi, plo, ncols, 0};
}

template <typename T, int N, int MODE, bool PBLK = false, int L = Tile<T>::L>
hipError_t launch_strided(const StridedArgs<T>& a0, const PlanView<T>& pv, hipStream_t s) {
    StridedArgs<T> a = a0;
    a.ncb = (a.ncols + L - 1) / L;
    // the kernel addresses a tile as uniform pointer + 32-bit per-lane byte
    // offset (row part of thread j plus a column < L): keep it in range
    const int jmax = PlanInfo<N>::TPL - 1;
    const int64_t prow = PBLK ? (int64_t)(jmax >> 3) * a.phi + (int64_t)(jmax & 7) * a.plo : (int64_t)jmax * a.pstride;
    if (a.ncols < 1 || (prow + L) * (int64_t)sizeof(cx<T>) >= (int64_t)1 << 32) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)(N * a.ncb);
    k_strided<T, N, MODE, L, PBLK><<<grid, L * PlanInfo<N>::TPL, 0, s>>>(a, pv);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::noise(const PlanView<T>& pv, uint64_t seed, uint32_t stream_id, T* w, hipStream_t s) {
    const uint64_t n3 = (uint64_t)pv.n * pv.n * pv.n;
    const uint64_t groups = n3 / 4;
    k_noise<T><<<capped_grid(groups, 256), 256, 0, s>>>(w, groups, seed, stream_id);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::fft_forward(const PlanView<T>& pv, const T* in, cx<T>* out, hipStream_t s) {
    return dispatch_n(pv.n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        constexpr int M = N / 2, L = Tile<T>::L;
        constexpr int64_t R = M + 1;  // row length of the plain half spectrum
        k_zfwd<T, N, false, true, false><<<N * N / L, L * PlanInfo<M>::TPL, 0, s>>>(in, out, pv.tw, 0, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // axis 1: o = k0, rows k1;  axis 0: o = k1, rows k0
        e = launch_strided<T, N, SMODE_FWD>(strided_args<T>(out, nullptr, out, nullptr, nullptr, N * R, 0, 0, R, 0, 0, M + 1),
                                           pv, s);
        if (e != hipSuccess) return e;
        return launch_strided<T, N, SMODE_FWD>(strided_args<T>(out, nullptr, out, nullptr, nullptr, R, 0, 0, N * R, 0, 0, M + 1),
                                              pv, s);
    });
}

template <typename T>
hipError_t Ops<T>::fft_inverse(const PlanView<T>& pv, const cx<T>* in, T* out, cx<T>* work, hipStream_t s) {
    return dispatch_n(pv.n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        constexpr int M = N / 2, L = Tile<T>::L;
        constexpr int64_t R = M + 1;
        hipError_t e = launch_strided<T, N, SMODE_INV>(
            strided_args<T>(in, nullptr, work, nullptr, nullptr, R, 0, 0, N * R, 0, 0, M + 1), pv, s);
        if (e != hipSuccess) return e;
        e = launch_strided<T, N, SMODE_INV>(
            strided_args<T>(work, nullptr, work, nullptr, nullptr, N * R, 0, 0, R, 0, 0, M + 1), pv, s);
        if (e != hipSuccess) return e;
        const T scale = (T)(1.0 / ((double)N * (double)N * (double)N));
        k_zinv<T, N, 0, false><<<dim3(N * N / L, 1), L * PlanInfo<M>::TPL, 0, s>>>(
            work, work, work, M + 1, out, scale, pv, ZelArgs{nullptr, nullptr, nullptr});
        return hipGetLastError();
    });
}

template <typename T>
hipError_t Ops<T>::filter(const PlanView<T>& pv, const cx<T>* w, cx<T>* psi, cx<T>* delta, hipStream_t s) {
    const int n = pv.n;
    const uint64_t total = (uint64_t)n * n * (n / 2 + 1);
    const T scale = (T)((double)n * (double)n * (double)n);
    const T kf = (T)(2.0 * kPi / pv.box);
    k_filter<T><<<capped_grid(total, 256), 256, 0, s>>>(w, psi, delta, n, scale, kf, pv.tau);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::zeldovich(const PlanView<T>& pv, const T* psi, float* pos, float* vel, hipStream_t s) {
    const uint64_t n3 = (uint64_t)pv.n * pv.n * pv.n;
    k_zeldovich<T><<<capped_grid(3 * n3, 256), 256, 0, s>>>(psi, pos, vel, pv);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::make_ic(const PlanView<T>& pv, uint64_t seed, float* pos, float* vel, T* psi, cx<T>* work,
                           hipStream_t s, hipEvent_t* ev) {
    return dispatch_n(pv.n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        constexpr int M = N / 2, L = Tile<T>::L;
        const size_t hsz = (size_t)N * N * M;
        cx<T>* b0 = work;
        cx<T>* b1 = work + hsz;
        cx<T>* b2 = work + 2 * hsz;
        hipError_t e;
#define GG_MARK(i) \
    if (ev && (e = hipEventRecord(ev[i], s)) != hipSuccess) return e;
        // spectra rows are blocked: row ((m0 / 8) N + k1) 8 + m0 % 8 holds k2 in [0, M)
        const int64_t H = (int64_t)8 * N * M;  // one m0 / 8 slab
        GG_MARK(0)
        k_zfwd<T, N, true, false, true><<<N * N / L, L * PlanInfo<M>::TPL, 0, s>>>(nullptr, b0, pv.tw, seed, 0u);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        GG_MARK(1)
        // P2: axis 1, o = m0
        e = launch_strided<T, N, SMODE_FWD>(strided_args<T>(b0, nullptr, b0, nullptr, nullptr, H, M, 3, 8 * M, 0, 0, M),
                                           pv, s);
        if (e != hipSuccess) return e;
        GG_MARK(2)
        // P3: axis 0, o = k1; W~ (b0) -> F (b1), G (b2)
        e = launch_strided<T, N, SMODE_XFILT, true>(strided_args<T>(b0, nullptr, b1, b2, nullptr, 8 * M, 0, 0, 0, H, M, M),
                                                   pv, s);
        if (e != hipSuccess) return e;
        GG_MARK(3)
        // P4: axis 1, o = m0; F (b1) -> A (b1), G (b2) -> B (b0), C (b2)
        e = launch_strided<T, N, SMODE_YINV3>(strided_args<T>(b1, b2, b1, b0, b2, H, M, 3, 8 * M, 0, 0, M), pv, s);
        if (e != hipSuccess) return e;
        GG_MARK(4)
        k_zinv<T, N, 1, true><<<dim3(N * N / L, 3), L * PlanInfo<M>::TPL, 0, s>>>(b1, b0, b2, M, nullptr, (T)1, pv,
                                                                                  ZelArgs{pos, vel, psi});
        if ((e = hipGetLastError()) != hipSuccess) return e;
        GG_MARK(5)
#undef GG_MARK
        return hipSuccess;
    });
}

template <typename T>
hipError_t Ops<T>::tau_table(T* tau, int64_t ntau, int n, double box, double amp_growth2, double gamma, double n_s,
                             hipStream_t s) {
    k_tau<T><<<capped_grid((uint64_t)ntau, 256), 256, 0, s>>>(tau, ntau, n, box, amp_growth2, gamma, n_s);
    return hipGetLastError();
}

}  // namespace gg
