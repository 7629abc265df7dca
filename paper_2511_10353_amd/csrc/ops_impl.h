// Definitions of Ops<T>: grid shapes and the pass sequence of the fused path.
#pragma once
#include <type_traits>

#include "cosmo_dev.h"
#include "diag.h"
#include "refine.h"
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
        case 96: return f(std::integral_constant<int, 96>{});
        case 128: return f(std::integral_constant<int, 128>{});
        case 160: return f(std::integral_constant<int, 160>{});
        case 192: return f(std::integral_constant<int, 192>{});
        case 256: return f(std::integral_constant<int, 256>{});
        case 512: return f(std::integral_constant<int, 512>{});
        case 1024: return f(std::integral_constant<int, 1024>{});
        default: return hipErrorInvalidValue;
    }
}

// Lines per work-group of the fused path's axis-2 passes.  Their rows are
// contiguous, so L only sets the LDS tile (and with it how many work-groups
// share a compute unit).
#ifndef GG_ZLINES
#define GG_ZLINES 16
#endif
template <typename T, int N>
struct ZLines {
    static constexpr int L = (GG_ZLINES < Tile<T>::L ? GG_ZLINES : Tile<T>::L) <= (N * N / 8)
                                 ? (GG_ZLINES < Tile<T>::L ? GG_ZLINES : Tile<T>::L)
                                 : Tile<T>::L;
};

// Lines per work-group of the first pass (noise + axis-2 transform): its LDS
// tile is kept to GG_P1_LDS bytes.  Sized so that a work-group of it would fit
// on a compute unit beside one of the axis-1 pass (128 KB of LDS at N = 1024);
// that sharing never paid when measured, and with the float path's 2 KB
// logarithm table beside the tile the two no longer fit together.
#ifndef GG_P1_LDS
#define GG_P1_LDS 32768
#endif
template <typename T, int N>
struct P1Lines {
    static constexpr int fit = GG_P1_LDS / (int)((N / 2) * sizeof(cx<T>));
    static constexpr int L = fit >= ZLines<T, N>::L ? ZLines<T, N>::L : (fit >= 1 ? fit : 1);
};

// Runs f with the compile-time line count of an axis-2 pass chosen at run
// time: `want` (0 = dflt) must be the full or the half tile.
template <typename T, int N, typename F>
hipError_t with_lines(int want, int dflt, F&& f) {
    constexpr int LF = ZLines<T, N>::L;
    constexpr int LH = LF / 2 >= 1 ? LF / 2 : 1;
    const int l = want ? want : dflt;
    if (l == LF) return f(std::integral_constant<int, LF>{});
    if (l == LH) return f(std::integral_constant<int, LH>{});
    return hipErrorInvalidValue;
}

inline unsigned capped_grid(uint64_t work, unsigned block) {
    uint64_t g = (work + block - 1) / block;
    const uint64_t cap = 256ull * 64ull;
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

template <typename T>
StridedArgs<T> strided_args(const cx<T>* in0, const cx<T>* in1, cx<T>* out0, cx<T>* out1, cx<T>* out2, int64_t ohi,
                            int64_t olo, int oshift, int64_t pstride, int64_t phi, int64_t plo, int ncols,
                            const cx<T>* in2 = nullptr) {
    return StridedArgs<T>{in0, in1, in2, out0, out1, out2, ohi, olo, oshift, pstride, phi, plo, ncols, 0, 0, 0, 2, 0};
}

// Launches tiles o in [o0, o0 + no) x column blocks [cb0, cb0 + nb) (nb = 0:
// all column blocks; no = 0: all N outer indices).
template <typename T, int N, int MODE, bool PBLK = false, int L = Tile<T>::L>
hipError_t launch_strided(const StridedArgs<T>& a0, const PlanView<T>& pv, hipStream_t s, int o0 = 0, int no = 0,
                          int cb0 = 0, int nb = 0, int nfields = 1) {
    StridedArgs<T> a = a0;
    const int ncb_all = (a.ncols + L - 1) / L;
    if (nb == 0) nb = ncb_all;
    if (no == 0) no = N;
    if (o0 < 0 || no < 1 || o0 + no > N || cb0 < 0 || nb < 1 || cb0 + nb > ncb_all) return hipErrorInvalidValue;
    a.ncb = nb;
    a.cb0 = cb0;
    a.o0 = o0;
    // the kernel addresses a tile as uniform pointer + 32-bit per-lane byte
    // offset (row part of thread j plus a column < L): keep it in range
    const int jmax = PlanInfo<N>::TPL - 1;
    const int64_t prow = PBLK ? (int64_t)(jmax >> 3) * a.phi + (int64_t)(jmax & 7) * a.plo : (int64_t)jmax * a.pstride;
    if (a.ncols < 1 || (prow + L) * (int64_t)sizeof(cx<T>) >= (int64_t)1 << 32) return hipErrorInvalidValue;
    if (nfields < 1 || (nfields > 1 && a.cstride <= 0)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(no * nb), (unsigned)nfields);
    k_strided<T, N, MODE, L, PBLK><<<grid, L * PlanInfo<N>::TPL, 0, s>>>(a, pv);
    return hipGetLastError();
}

// P3 of float plans: the persistent k_xfilt over column blocks [cb0, cb0 + nb)
// of every outer index (blocked rows), with launch_strided's checks; one
// work-group per compute unit (cus = 0: one per tile).
template <typename T, int N>
hipError_t launch_xfilt(const StridedArgs<T>& a0, const PlanView<T>& pv, hipStream_t s, int cb0, int nb, int cus) {
    constexpr int L = Tile<T>::L;
    StridedArgs<T> a = a0;
    const int ncb_all = (a.ncols + L - 1) / L;
    if (cb0 < 0 || nb < 1 || cb0 + nb > ncb_all) return hipErrorInvalidValue;
    a.ncb = nb;
    a.cb0 = cb0;
    a.o0 = 0;
    const int jmax = PlanInfo<N>::TPL - 1;
    const int64_t prow = (int64_t)(jmax >> 3) * a.phi + (int64_t)(jmax & 7) * a.plo;
    if (a.ncols < 1 || (prow + L) * (int64_t)sizeof(cx<T>) >= (int64_t)1 << 32) return hipErrorInvalidValue;
    const int ntiles = N * nb;
    const int grid = cus > 0 && cus < ntiles ? cus : ntiles;
    k_xfilt<T, N, L><<<grid, L * PlanInfo<N>::TPL, 0, s>>>(a, pv, ntiles);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::noise(const PlanView<T>& pv, uint64_t seed, uint32_t stream_id, T* w, hipStream_t s) {
    const uint64_t n3 = (uint64_t)pv.n * pv.n * pv.n;
    k_noise<T><<<capped_grid(n3, 256), 256, 0, s>>>(w, n3, seed, stream_id, pv.lntab);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::fft_forward(const PlanView<T>& pv, const T* in, cx<T>* out, hipStream_t s) {
    return dispatch_n(pv.n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        constexpr int M = N / 2, L = Tile<T>::L;
        constexpr int64_t R = M + 1;  // row length of the plain half spectrum
        const ZSrc<T> zs{in, nullptr, nullptr, nullptr, 0.0, 0, nullptr, nullptr};
        k_zfwd<T, N, ZSRC_REAL, true, false><<<N * N / L, L * PlanInfo<M>::TPL, 0, s>>>(zs, out, pv.tw, 0, 0, 0);
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
        k_zinv<T, N, false><<<N * N / L, L * PlanInfo<M>::TPL, 0, s>>>(work, M + 1, M + 1, 0, out, scale, pv);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t Ops<T>::filter(const PlanView<T>& pv, const cx<T>* w, cx<T>* psi, cx<T>* delta, hipStream_t s) {
    const int n = pv.n;
    const uint64_t total = (uint64_t)n * n * (n / 2 + 1);
    const T scale = (T)((double)n * (double)n * (double)n);
    const T kf = (T)(2.0 * kPi / pv.box);
    k_filter<T><<<capped_grid(total, 256), 256, 0, s>>>(w, psi, delta, n, scale, kf, pv);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::zeldovich(const PlanView<T>& pv, const T* psi, float* pos, float* vel, hipStream_t s) {
    const unsigned bz = pv.n < 256 ? (unsigned)((pv.n + 63) / 64 * 64) : 256u;
    k_zeldovich<T><<<dim3((unsigned)(pv.n * pv.n), (unsigned)((pv.n + bz - 1) / bz), 3), bz, 0, s>>>(psi, pos, vel, pv);
    return hipGetLastError();
}

template <typename T>
void Ops<T>::tile_options(int n, int& full, int& half, int& p1_default, int& z_default) {
    full = half = p1_default = z_default = 0;  // left at 0 for a size without a plan
    (void)dispatch_n(n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        full = ZLines<T, N>::L;
        half = full / 2 >= 1 ? full / 2 : 1;
        p1_default = P1Lines<T, N>::L;
        z_default = ZLines<T, N>::L;
        return hipSuccess;
    });
}

template <typename T>
int Ops<T>::max_chunks(int n) {
    // axis-0 slabs of whole 8-row groups and k2 chunks of whole column blocks;
    // measured best at 1024^3: 4 chunks (float), 2 (double)
    const int slabs = n / 8, cblocks = (n / 2) / Tile<T>::L;
    const int cap = sizeof(T) == 4 ? 4 : 2;
    int c = 1;
    while (c < cap && slabs % (2 * c) == 0 && cblocks % (2 * c) == 0 && n >= 256) c *= 2;
    return c;
}

template <typename T>
hipError_t Ops<T>::make_ic(const PlanView<T>& pv, uint64_t seed, float* pos, float* vel, T* psi, cx<T>* work,
                           const ExecCtx& x) {
    return fused_forward(pv, nullptr, seed, pos, vel, psi, work, x);
}

template <typename T>
hipError_t Ops<T>::make_ic_from_noise(const PlanView<T>& pv, const T* w, float* pos, float* vel, T* psi, cx<T>* work,
                                      const ExecCtx& x) {
    return fused_forward(pv, w, 0, pos, vel, psi, work, x);
}

template <typename T>
hipError_t Ops<T>::fused_forward(const PlanView<T>& pv, const T* w, uint64_t seed, float* pos, float* vel, T* psi,
                                 cx<T>* work, const ExecCtx& x) {
    return dispatch_n(pv.n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        constexpr int M = N / 2;
        constexpr int LZ = ZLines<T, N>::L;
        const int NC = (x.b && x.sync) ? x.nchunk : 1;
        if (NC < 1 || (N / 8) % NC != 0 || ((M + Tile<T>::L - 1) / Tile<T>::L) % NC != 0) return hipErrorInvalidValue;
        const hipStream_t sa = x.a;
        const hipStream_t sb = NC > 1 ? x.b : x.a;
        const size_t hsz = (size_t)N * N * M;
        cx<T>* b0 = work;
        cx<T>* b1 = work + hsz;
        cx<T>* b2 = work + 2 * hsz;
        hipError_t e = hipSuccess;
        int launch = 0;
        auto mark = [&](hipStream_t st, int which) -> hipError_t {
            return x.tev ? hipEventRecord(x.tev[2 * launch + which], st) : hipSuccess;
        };
#define GG_TRY(expr) \
    if ((e = (expr)) != hipSuccess) return e;
        // spectra rows are blocked: row ((m0 / 8) N + k1) 8 + m0 % 8 holds k2 in [0, M)
        const int64_t H = (int64_t)8 * N * M;  // one m0 / 8 slab
        StridedArgs<T> a2 = strided_args<T>(b0, nullptr, b0, nullptr, nullptr, H, M, 3, 8 * M, 0, 0, M);
        const StridedArgs<T> a3 = strided_args<T>(b0, nullptr, b1, b2, nullptr, 8 * M, 0, 0, 0, H, M, M);
        StridedArgs<T> a4 = strided_args<T>(b1, b2, b1, b0, b2, H, M, 3, 8 * M, 0, 0, M);
        // XCD tile orders measured best at 1024^3: P2 and P4 one range per XCD,
        // P3 pairs
        a2.xgroup = 0;
        a4.xgroup = 0;
        const int xh = (N / 8) / NC;                           // m0 / 8 values per slab
        const int nb = ((M + Tile<T>::L - 1) / Tile<T>::L) / NC;  // column blocks per chunk
        if (NC > 1) {
            GG_TRY(hipEventRecord(x.sync[0], sa))
            GG_TRY(hipStreamWaitEvent(sb, x.sync[0], 0))
        }
        // P1 on slab s (rows of m0 in [8 xh s, 8 xh (s+1))), then P2 on the same slab
        for (int s = 0; s < NC; ++s) {
            launch = s;
            const uint64_t row0 = (uint64_t)s * xh * 8 * N;
            GG_TRY(mark(sa, 0))
            GG_TRY((with_lines<T, N>(x.p1_lines, P1Lines<T, N>::L, [&](auto lc) -> hipError_t {
                constexpr int L1 = decltype(lc)::value;
                const unsigned blocks = (unsigned)((uint64_t)xh * 8 * N / L1);
                if (w) {
                    const ZSrc<T> zs{w, nullptr, nullptr, nullptr, 0.0, 0, nullptr, nullptr};
                    k_zfwd<T, N, ZSRC_REAL, false, true, L1><<<blocks, L1 * PlanInfo<M>::TPL, 0, sa>>>(zs, b0, pv.tw, 0,
                                                                                                      0u, row0);
                } else {
                    ZSrc<T> zs{nullptr, nullptr, nullptr, nullptr, 0.0, 0, nullptr, nullptr};
                    zs.lntab = pv.lntab;
                    k_zfwd<T, N, ZSRC_NOISE, false, true, L1><<<blocks, L1 * PlanInfo<M>::TPL, 0, sa>>>(zs, b0, pv.tw,
                                                                                                       seed, 0u, row0);
                }
                return hipGetLastError();
            })))
            GG_TRY(mark(sa, 1))
            if (NC > 1) {
                GG_TRY(hipEventRecord(x.sync[1 + s], sa))
                GG_TRY(hipStreamWaitEvent(sb, x.sync[1 + s], 0))
            }
            launch = NC + s;
            GG_TRY(mark(sb, 0))
            GG_TRY((launch_strided<T, N, SMODE_FWD>(a2, pv, sb, 8 * xh * s, 8 * xh)))
            GG_TRY(mark(sb, 1))
        }
        if (NC > 1) {
            GG_TRY(hipEventRecord(x.sync[NC + 1], sb))
            GG_TRY(hipStreamWaitEvent(sa, x.sync[NC + 1], 0))
        }
        // P3 on k2 chunk q (all k1), then P4 on the same chunk (all m0)
        for (int q = 0; q < NC; ++q) {
            launch = 2 * NC + q;
            GG_TRY(mark(sa, 0))
            if constexpr (std::is_same_v<T, float>) {
                GG_TRY((launch_xfilt<T, N>(a3, pv, sa, nb * q, nb, x.cus)))
            } else {
                GG_TRY((launch_strided<T, N, SMODE_XFILT, true>(a3, pv, sa, 0, 0, nb * q, nb)))
            }
            GG_TRY(mark(sa, 1))
            if (NC > 1) {
                GG_TRY(hipEventRecord(x.sync[NC + 2 + q], sa))
                GG_TRY(hipStreamWaitEvent(sb, x.sync[NC + 2 + q], 0))
            }
            launch = 3 * NC + q;
            GG_TRY(mark(sb, 0))
            GG_TRY((launch_strided<T, N, SMODE_YINV3>(a4, pv, sb, 0, 0, nb * q, nb)))
            GG_TRY(mark(sb, 1))
        }
        if (NC > 1) {
            GG_TRY(hipEventRecord(x.sync[2 * NC + 2], sb))
            GG_TRY(hipStreamWaitEvent(sa, x.sync[2 * NC + 2], 0))
        }
        launch = 4 * NC;
        GG_TRY(mark(sa, 0))
        GG_TRY((with_lines<T, N>(x.z_lines, LZ, [&](auto lc) -> hipError_t {
            constexpr int L5 = decltype(lc)::value;
            // components 0, 1, 2 are in b1, b0, b2 (P4's outputs)
            const int ntiles = 3 * (N * N / L5);
            const int grid = x.cus > 0 && 16 * x.cus < ntiles ? 16 * x.cus : ntiles;
            const dim3 gd(grid), bd(L5 * PlanInfo<M>::TPL);
            const ZelArgs za{pos, vel, psi};
            if (pos && psi) k_zel<T, N, L5, true, true><<<gd, bd, 0, sa>>>(b1, b0, b2, pv, za, ntiles);
            else if (pos) k_zel<T, N, L5, true, false><<<gd, bd, 0, sa>>>(b1, b0, b2, pv, za, ntiles);
            else if (psi) k_zel<T, N, L5, false, true><<<gd, bd, 0, sa>>>(b1, b0, b2, pv, za, ntiles);
            return hipGetLastError();
        })))
        GG_TRY(mark(sa, 1))
#undef GG_TRY
        return hipSuccess;
    });
}

template <typename T>
hipError_t Ops<T>::adjoint(const PlanView<T>& pv, const T* gpsi, const float* gpos, const float* gvel, const T* psi,
                           double* g_log_amp, T* gw, cx<T>* work, hipStream_t s) {
    return dispatch_n(pv.n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        constexpr int M = N / 2;
        constexpr int LZ = ZLines<T, N>::L;
        const size_t hsz = (size_t)N * N * M;
        cx<T>* b0 = work;
        cx<T>* b1 = work + hsz;
        cx<T>* b2 = work + 2 * hsz;
        // d loss / d log A = (1/2) sum g psi (psi scales as sqrt(A)): A1 leaves one
        // partial sum per work-group in gw, which A5 overwrites later
        const bool dot = g_log_amp && psi;
        const uint32_t nblk = (uint32_t)(N * N / LZ);
        static_assert(3 * (N * N / LZ) * sizeof(double) <= (size_t)N * N * N * sizeof(T), "partials must fit in gw");
        double* part = reinterpret_cast<double*>(gw);
        const ZSrc<T> zs{nullptr, gpsi, gpos, gvel, pv.vfac, (uint64_t)hsz, dot ? psi : nullptr, dot ? part : nullptr};
        hipError_t e;
#define GG_TRY(expr) \
    if ((e = (expr)) != hipSuccess) return e;
        // A1: axis-2 r2c of the three gradient components -> b0, b1, b2 (blocked rows)
        k_zfwd<T, N, ZSRC_GRAD, false, true, LZ><<<dim3(nblk, 3), LZ * PlanInfo<M>::TPL, 0, s>>>(zs, b0, pv.tw, 0,
                                                                                                  0u, 0);
        GG_TRY(hipGetLastError())
        if (dot) {
            GG_TRY(launch_dot_final(part, 3 * nblk, 0.5, g_log_amp, s))
        }
        // A2: axis-1 forwards of the three components: Y0 -> b0 and
        // Z = s1 Y1 + s2 Y2 -> b1 (one contiguous tile range per XCD, as P2)
        const int64_t H = (int64_t)8 * N * M;
        StridedArgs<T> a2 = strided_args<T>(b0, nullptr, b0, nullptr, nullptr, H, M, 3, 8 * M, 0, 0, M);
        a2.xgroup = 0;
        GG_TRY((launch_strided<T, N, SMODE_FWD>(a2, pv, s)))
        StridedArgs<T> a2z = strided_args<T>(b1, b2, b1, nullptr, nullptr, H, M, 3, 8 * M, 0, 0, M);
        a2z.xgroup = 0;
        GG_TRY((launch_strided<T, N, SMODE_YADJ>(a2z, pv, s)))
        // A3: axis-0 forwards of Y0 and Z, -i tau (s0 X0 + Z'), axis-0 inverse -> b0
        GG_TRY((launch_strided<T, N, SMODE_XADJ, true>(
            strided_args<T>(b0, b1, b0, nullptr, nullptr, 8 * M, 0, 0, 0, H, M, M), pv, s)))
        // A4: axis-1 inverse
        StridedArgs<T> a4 = strided_args<T>(b0, nullptr, b0, nullptr, nullptr, H, M, 3, 8 * M, 0, 0, M);
        a4.xgroup = 0;
        GG_TRY((launch_strided<T, N, SMODE_INV>(a4, pv, s)))
        // A5: axis-2 c2r -> d loss / d W (the 1/N^3 is inside tau)
        k_zinv<T, N, true, LZ><<<N * N / LZ, LZ * PlanInfo<M>::TPL, 0, s>>>(b0, M, M, 0, gw, (T)1, pv);
        GG_TRY(hipGetLastError())
#undef GG_TRY
        return hipSuccess;
    });
}

template <typename T>
hipError_t Ops<T>::density(const PlanView<T>& pv, uint64_t seed, const T* w, T* delta, cx<T>* work, hipStream_t s) {
    return dispatch_n(pv.n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        constexpr int M = N / 2;
        constexpr int LZ = ZLines<T, N>::L;
        constexpr int L1 = P1Lines<T, N>::L;
        cx<T>* b0 = work;
        hipError_t e;
#define GG_TRY(expr) \
    if ((e = (expr)) != hipSuccess) return e;
        const int64_t H = (int64_t)8 * N * M;
        ZSrc<T> zs{w, nullptr, nullptr, nullptr, 0.0, 0, nullptr, nullptr};
        zs.lntab = pv.lntab;
        if (w)
            k_zfwd<T, N, ZSRC_REAL, false, true, L1><<<N * N / L1, L1 * PlanInfo<M>::TPL, 0, s>>>(zs, b0, pv.tw, 0, 0u, 0);
        else
            k_zfwd<T, N, ZSRC_NOISE, false, true, L1><<<N * N / L1, L1 * PlanInfo<M>::TPL, 0, s>>>(zs, b0, pv.tw, seed,
                                                                                                 0u, 0);
        GG_TRY(hipGetLastError())
        GG_TRY((launch_strided<T, N, SMODE_FWD>(strided_args<T>(b0, nullptr, b0, nullptr, nullptr, H, M, 3, 8 * M, 0, 0, M),
                                                pv, s)))
        GG_TRY((launch_strided<T, N, SMODE_XDELTA, true>(
            strided_args<T>(b0, nullptr, b0, nullptr, nullptr, 8 * M, 0, 0, 0, H, M, M), pv, s)))
        GG_TRY((launch_strided<T, N, SMODE_INV>(strided_args<T>(b0, nullptr, b0, nullptr, nullptr, H, M, 3, 8 * M, 0, 0, M),
                                                pv, s)))
        k_zinv<T, N, true, LZ><<<N * N / LZ, LZ * PlanInfo<M>::TPL, 0, s>>>(b0, M, M, 0, delta, (T)1, pv);
        GG_TRY(hipGetLastError())
#undef GG_TRY
        return hipSuccess;
    });
}

template <typename T>
hipError_t Ops<T>::power_spectrum(const PlanView<T>& pv, const T* field, int nbins, double* pk, double* kmean,
                                  double* counts, cx<T>* work, size_t work_bytes, hipStream_t s) {
    const int n = pv.n;
    const size_t spec_bytes = (size_t)n * n * (n / 2 + 1) * sizeof(cx<T>);
    const size_t part_off = (spec_bytes + 255) / 256 * 256;
    if (nbins < 1 || nbins > kPkMaxBins || part_off >= work_bytes) return hipErrorInvalidValue;
    // work-groups: a power of two dividing the N^2 rows, at most 1024, whose
    // partial sums fit behind the spectrum
    const size_t per_block = (size_t)3 * nbins * sizeof(double);
    int64_t nblocks = 1;
    while (nblocks * 2 <= 1024 && nblocks * 2 <= (int64_t)n * n && (size_t)(nblocks * 2) * per_block <= work_bytes - part_off)
        nblocks *= 2;
    if ((size_t)nblocks * per_block > work_bytes - part_off) return hipErrorInvalidValue;
    hipError_t e = fft_forward(pv, field, work, s);
    if (e != hipSuccess) return e;
    double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(work) + part_off);
    const size_t shmem = (size_t)3 * nbins * sizeof(double) + 3 * kPkThreads * sizeof(double) + kPkThreads * sizeof(int);
    k_pk_rows<T><<<(unsigned)nblocks, kPkThreads, shmem, s>>>(work, n, nbins, (int)((int64_t)n * n / nblocks), part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const double n3 = (double)n * n * n;
    k_pk_final<T><<<(nbins + 255) / 256, 256, 0, s>>>(part, (int)nblocks, nbins, pv.box * pv.box * pv.box / (n3 * n3),
                                                      2.0 * 3.14159265358979323846 / pv.box, pk, kmean, counts);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::field_stats(const T* field, uint64_t count, double* out, double* scratch, int nblocks,
                               hipStream_t s) {
    if (nblocks < 1 || count == 0) return hipErrorInvalidValue;
    k_stats_partial<T, false><<<nblocks, kStatThreads, 0, s>>>(field, count, nullptr, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_stats_final<T, false><<<1, 1, 0, s>>>(scratch, nblocks, count, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_stats_partial<T, true><<<nblocks, kStatThreads, 0, s>>>(field, count, out, scratch);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_stats_final<T, true><<<1, 1, 0, s>>>(scratch, nblocks, count, out);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::refine(int variant, const T* parent, int n_parent, const int origin[3], int count, uint64_t seed,
                          uint32_t stream_id, T* child, hipStream_t s) {
    auto run = [&](auto vc) -> hipError_t {
        constexpr int VAR = decltype(vc)::value;
        constexpr int NL = RefineBasis<VAR>::NL;
        if (count < NL || count % NL || count > n_parent) return hipErrorInvalidValue;
        for (int a = 0; a < 3; ++a)
            if (origin[a] < 0 || origin[a] >= n_parent) return hipErrorInvalidValue;
        const int P = count / NL;
        const uint64_t np = (uint64_t)P * P * P;
        k_refine<T, VAR><<<(unsigned)((np + kRefineThreads - 1) / kRefineThreads), kRefineThreads, 0, s>>>(
            parent, n_parent, origin[0], origin[1], origin[2], P, seed, stream_id, child);
        return hipGetLastError();
    };
    switch (variant) {
        case REFINE_HR: return run(std::integral_constant<int, REFINE_HR>{});
        case REFINE_3: return run(std::integral_constant<int, REFINE_3>{});
        case REFINE_4: return run(std::integral_constant<int, REFINE_4>{});
        case REFINE_LINEAR: return run(std::integral_constant<int, REFINE_LINEAR>{});
        case REFINE_SINE: return run(std::integral_constant<int, REFINE_SINE>{});
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t Ops<T>::cic_add(const T* src, int n_src, int num, int den, const int origin[3], T* dst, int n_dst,
                           hipStream_t s) {
    if (n_src < 1 || n_dst < 1 || num < 1 || den < 1) return hipErrorInvalidValue;
    for (int a = 0; a < 3; ++a)
        if (origin[a] < 0 || origin[a] >= n_src) return hipErrorInvalidValue;
    if (n_dst > 4096) return hipErrorInvalidValue;
    const unsigned bc = n_dst < 256 ? (unsigned)((n_dst + 63) / 64 * 64) : 256u;
    k_cic_add<T, false><<<dim3((unsigned)(n_dst * n_dst), (unsigned)((n_dst + bc - 1) / bc)), bc, 0, s>>>(
        src, n_src, num, den, origin[0], origin[1], origin[2], dst, n_dst, PlanView<T>{}, nullptr, nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::cic_add_zel(const T* src, int n_src, int num, int den, const int origin[3], T* dst,
                               const PlanView<T>& pv, float* pos, float* vel, hipStream_t s) {
    const int n_dst = pv.n;
    if (n_src < 1 || n_dst < 1 || num < 1 || den < 1) return hipErrorInvalidValue;
    for (int a = 0; a < 3; ++a)
        if (origin[a] < 0 || origin[a] >= n_src) return hipErrorInvalidValue;
    if (n_dst > 4096) return hipErrorInvalidValue;
    const unsigned bc = n_dst < 256 ? (unsigned)((n_dst + 63) / 64 * 64) : 256u;
    k_cic_add<T, true><<<dim3((unsigned)(n_dst * n_dst), (unsigned)((n_dst + bc - 1) / bc)), bc, 0, s>>>(
        src, n_src, num, den, origin[0], origin[1], origin[2], dst, n_dst, pv, pos, vel);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::lowpass3(const PlanView<T>& pv0, const T* field, int n2_max, int deconv, T* out, cx<T>* work,
                            hipStream_t s) {
    const int n = pv0.n;
    const uint64_t n3 = (uint64_t)n * n * n;
    // modes |n_j| <= kmax survive the window n^2 < n2_max: the half spectrum
    // is kept to kc columns (whole column blocks); without room for that, the
    // full transform per field
    int kmax = 0;
    while ((int64_t)(kmax + 1) * (kmax + 1) < (int64_t)n2_max) ++kmax;
    constexpr int L = Tile<T>::L;
    const int kc = (kmax + 1 + L - 1) / L * L;
    if (n2_max <= 0 || kc >= n / 2) {
        for (int j = 0; j < 3; ++j) {
            const hipError_t e = lowpass(pv0, field + j * n3, n2_max, deconv, out + j * n3, work, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    PlanView<T> pv = pv0;
    pv.n2_lo = 0;
    pv.n2_hi = n2_max;
    pv.deconv = deconv ? 1 : 0;
    return dispatch_n(n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        constexpr int M = N / 2;
        const int64_t fs = (int64_t)N * N * kc;  // one pruned spectrum
        ZSrc<T> zs{field, nullptr, nullptr, nullptr, 0.0, (uint64_t)fs, nullptr, nullptr};
        zs.wstride_comp = n3;
        zs.kout = kc;
        k_zfwd<T, N, ZSRC_REAL, false, false><<<dim3(N * N / L, 3), L * PlanInfo<M>::TPL, 0, s>>>(zs, work, pv.tw, 0, 0,
                                                                                                  0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // axis 1: o = m0 (rows m1, kc columns); axis 0: o = k1 (rows k0)
        StridedArgs<T> a1 = strided_args<T>(work, nullptr, work, nullptr, nullptr, (int64_t)N * kc, 0, 0, kc, 0, 0, kc);
        StridedArgs<T> a0 = strided_args<T>(work, nullptr, work, nullptr, nullptr, kc, 0, 0, (int64_t)N * kc, 0, 0, kc);
        a1.cstride = a0.cstride = fs;
        if ((e = launch_strided<T, N, SMODE_FWD>(a1, pv, s, 0, 0, 0, 0, 3)) != hipSuccess) return e;
        if ((e = launch_strided<T, N, SMODE_XWIN>(a0, pv, s, 0, 0, 0, 0, 3)) != hipSuccess) return e;
        if ((e = launch_strided<T, N, SMODE_INV>(a1, pv, s, 0, 0, 0, 0, 3)) != hipSuccess) return e;
        const T scale = (T)(1.0 / ((double)N * (double)N * (double)N));
        k_zinv<T, N, false><<<dim3(N * N / L, 3), L * PlanInfo<M>::TPL, 0, s>>>(work, kc, kc, (uint64_t)fs, out, scale,
                                                                               pv);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t Ops<T>::windowed_displacements(const PlanView<T>& pv0, const T* w, int n2_max, int deconv, T* psi,
                                          cx<T>* work, const ExecCtx& x) {
    const int n = pv0.n;
    int kmax = 0;
    while ((int64_t)(kmax + 1) * (kmax + 1) < (int64_t)n2_max) ++kmax;
    constexpr int L = Tile<T>::L;
    const int kc = (kmax + 1 + L - 1) / L * L;
    PlanView<T> pv = pv0;
    pv.n2_lo = 0;
    pv.n2_hi = n2_max;
    pv.deconv = deconv ? 1 : 0;
    if (n2_max <= 0 || kc >= n / 2) return make_ic_from_noise(pv, w, nullptr, nullptr, psi, work, x);
    const hipStream_t s = x.a;
    return dispatch_n(n, [&](auto nc) -> hipError_t {
        constexpr int N = decltype(nc)::value;
        constexpr int M = N / 2;
        const int64_t fs = (int64_t)N * N * kc;  // one pruned spectrum
        cx<T>* s0 = work;
        cx<T>* s1 = work + fs;
        cx<T>* s2 = work + 2 * fs;
        ZSrc<T> zs{w, nullptr, nullptr, nullptr, 0.0, 0, nullptr, nullptr};
        zs.kout = kc;
        k_zfwd<T, N, ZSRC_REAL, false, false><<<N * N / L, L * PlanInfo<M>::TPL, 0, s>>>(zs, s0, pv.tw, 0, 0, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // axis 1 forward; axis 0: F = IFFT(i s0 tau' W~), G = IFFT(i tau' W~) with
        // tau' the filter on the window; axis 1: A = IFFT(F), B = IFFT(s1 G),
        // C = IFFT(G); c2r of A, B and s2 C
        const StridedArgs<T> a1 = strided_args<T>(s0, nullptr, s0, nullptr, nullptr, (int64_t)N * kc, 0, 0, kc, 0, 0, kc);
        if ((e = launch_strided<T, N, SMODE_FWD>(a1, pv, s)) != hipSuccess) return e;
        const StridedArgs<T> a3 = strided_args<T>(s0, nullptr, s1, s2, nullptr, kc, 0, 0, (int64_t)N * kc, 0, 0, kc);
        if ((e = launch_strided<T, N, SMODE_XFILT>(a3, pv, s)) != hipSuccess) return e;
        const StridedArgs<T> a4 = strided_args<T>(s1, s2, s0, s1, s2, (int64_t)N * kc, 0, 0, kc, 0, 0, kc);
        if ((e = launch_strided<T, N, SMODE_YINV3>(a4, pv, s)) != hipSuccess) return e;
        k_zinv<T, N, false><<<dim3(N * N / L, 3), L * PlanInfo<M>::TPL, 0, s>>>(s0, kc, kc, (uint64_t)fs, psi, (T)1, pv,
                                                                               2);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t Ops<T>::lowpass(const PlanView<T>& pv, const T* field, int n2_max, int deconv, T* out, cx<T>* work,
                           hipStream_t s) {
    const int n = pv.n;
    const size_t hsz = (size_t)n * n * (n / 2 + 1);
    hipError_t e = fft_forward(pv, field, work, s);
    if (e != hipSuccess) return e;
    k_window<T><<<capped_grid(hsz, 256), 256, 0, s>>>(work, n, n2_max, deconv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return fft_inverse(pv, work, out, work + hsz, s);
}

template <typename T>
hipError_t Ops<T>::degrade(const PlanView<T>& pv, const T* fine, int factor, const double shift[3], T* out,
                           cx<T>* work, hipStream_t s) {
    const int n = pv.n;
    const uint64_t n3 = (uint64_t)n * n * n;
    const size_t hsz = (size_t)n * n * (n / 2 + 1);
    k_decimate<T><<<capped_grid(n3, 256), 256, 0, s>>>(fine, n, factor, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = fft_forward(pv, out, work, s)) != hipSuccess) return e;
    k_translate<T><<<capped_grid(hsz, 256), 256, 0, s>>>(work, n, shift[0], shift[1], shift[2]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return fft_inverse(pv, work, out, work + hsz, s);
}

template <typename T>
hipError_t Ops<T>::tau_table(T* tau, int64_t ntau, void* tauseg, int n, double box, double amp_growth2,
                             double gamma, double n_s, hipStream_t s) {
    k_tau<T><<<capped_grid((uint64_t)ntau, 256), 256, 0, s>>>(tau, ntau, n, box, amp_growth2, gamma, n_s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && tauseg) {
        if constexpr (sizeof(T) == 4)
            k_tauseg<T><<<(kTauSeg + 255) / 256, 256, 0, s>>>(static_cast<float4*>(tauseg), n, box, amp_growth2,
                                                               gamma, n_s);
        else
            k_tauseg64<T><<<(kTauSeg64 + 63) / 64, 64, 0, s>>>(static_cast<double*>(tauseg), n, box, amp_growth2,
                                                                gamma, n_s);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace gg
