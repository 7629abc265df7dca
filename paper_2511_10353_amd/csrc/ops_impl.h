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

template <typename T, int N, int MODE>
hipError_t launch_strided(const StridedArgs<T>& a0, const PlanView<T>& pv, hipStream_t s) {
    constexpr int L = Tile<T>::L;
    StridedArgs<T> a = a0;
    a.ncb = (a.ncols + L - 1) / L;
    const unsigned grid = (unsigned)(N * a.ncb);
    k_strided<T, N, MODE><<<grid, L * PlanInfo<N>::TPL, 0, s>>>(a, pv);
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
        k_zfwd<T, N, false, true><<<N * N / L, L * PlanInfo<M>::TPL, 0, s>>>(in, out, pv.tw, 0, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        StridedArgs<T> a{out, out, nullptr, nullptr, (int64_t)N * (M + 1), (int64_t)(M + 1), M + 1, 0};
        e = launch_strided<T, N, SMODE_FWD>(a, pv, s);
        if (e != hipSuccess) return e;
        a.ostride = M + 1;
        a.pstride = (int64_t)N * (M + 1);
        return launch_strided<T, N, SMODE_FWD>(a, pv, s);
    });
}

template <typename T>
hipError_t Ops<T>::fft_inverse(const PlanView<T>& pv, const cx<T>* in, T* out, cx<T>* work, hipStream_t s) {
    return dispatch_n(pv.n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        constexpr int M = N / 2, L = Tile<T>::L;
        StridedArgs<T> a{in, work, nullptr, nullptr, (int64_t)(M + 1), (int64_t)N * (M + 1), M + 1, 0};
        hipError_t e = launch_strided<T, N, SMODE_INV>(a, pv, s);
        if (e != hipSuccess) return e;
        a.src = work;
        a.ostride = (int64_t)N * (M + 1);
        a.pstride = M + 1;
        e = launch_strided<T, N, SMODE_INV>(a, pv, s);
        if (e != hipSuccess) return e;
        const T scale = (T)(1.0 / ((double)N * (double)N * (double)N));
        k_zinv<T, N, 0><<<dim3(N * N / L, 1), L * PlanInfo<M>::TPL, 0, s>>>(work, work, work, M + 1, out, scale, pv,
                                                                            ZelArgs{nullptr, nullptr, nullptr});
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
        GG_MARK(0)
        k_zfwd<T, N, true, false><<<N * N / L, L * PlanInfo<M>::TPL, 0, s>>>(nullptr, b0, pv.tw, seed, 0u);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        GG_MARK(1)
        StridedArgs<T> a{b0, b0, nullptr, nullptr, (int64_t)N * M, (int64_t)M, M, 0};
        if ((e = launch_strided<T, N, SMODE_FWD>(a, pv, s)) != hipSuccess) return e;
        GG_MARK(2)
        a = StridedArgs<T>{b0, b0, b1, nullptr, (int64_t)M, (int64_t)N * M, M, 0};
        if ((e = launch_strided<T, N, SMODE_XFILT>(a, pv, s)) != hipSuccess) return e;
        GG_MARK(3)
        a = StridedArgs<T>{b0, b0, b1, b2, (int64_t)N * M, (int64_t)M, M, 0};
        if ((e = launch_strided<T, N, SMODE_YINV3>(a, pv, s)) != hipSuccess) return e;
        GG_MARK(4)
        k_zinv<T, N, 1><<<dim3(N * N / L, 3), L * PlanInfo<M>::TPL, 0, s>>>(b0, b2, b1, M, nullptr, (T)1, pv,
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
