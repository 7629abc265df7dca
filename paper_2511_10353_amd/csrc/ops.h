// Host-side launchers of the kernels, per arithmetic type.  Declared here,
// defined (and explicitly instantiated) in gg_f32.hip and gg_f64.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.h"

namespace gg {

template <typename T>
struct PlanView;

// Lattice sizes the kernels are instantiated for: powers of two, and the
// uneven sizes 96 = 2^5 3, 160 = 2^5 5, 192 = 2^6 3 (mixed-radix plans).
constexpr bool supported_n(int n) {
    return n == 8 || n == 16 || n == 32 || n == 64 || n == 96 || n == 128 || n == 160 || n == 192 || n == 256 ||
           n == 512 || n == 1024;
}

// Launch context of the fused path.  With nchunk > 1 and an auxiliary stream,
// P1/P2 are pipelined over axis-0 slabs and P3/P4 over k2 column chunks: the
// first pass of each pair runs on the caller's stream, the second on the
// auxiliary one, each chunk waiting for its producer (events in sync[],
// 2 nchunk + 3 of them).  Passes with different limits (noise arithmetic vs
// memory traffic) then share the GPU.  tev (or null): 2 events per launch,
// launches ordered P1 chunks, P2 chunks, P3 chunks, P4 chunks, P5.
struct ExecCtx {
    hipStream_t a = nullptr;
    hipStream_t b = nullptr;
    hipEvent_t* sync = nullptr;
    int nchunk = 1;
    hipEvent_t* tev = nullptr;
    // lines per work-group of the first pass and of the last (particle) pass;
    // 0 = the built-in choice.  Each accepts the type's full LDS row of lines
    // (16 float, 8 double) or half of it.
    int p1_lines = 0;
    int z_lines = 0;
    // compute units of the device: the persistent passes (P3 for float
    // plans, P5) size their grids by it (0 = one work-group per tile)
    int cus = 0;
};

template <typename T>
struct Ops {
    static hipError_t noise(const PlanView<T>& pv, uint64_t seed, uint32_t stream_id, T* w, hipStream_t s);
    static hipError_t fft_forward(const PlanView<T>& pv, const T* in, cx<T>* out, hipStream_t s);
    static hipError_t fft_inverse(const PlanView<T>& pv, const cx<T>* in, T* out, cx<T>* work, hipStream_t s);
    static hipError_t filter(const PlanView<T>& pv, const cx<T>* w, cx<T>* psi, cx<T>* delta, hipStream_t s);
    static hipError_t zeldovich(const PlanView<T>& pv, const T* psi, float* pos, float* vel, hipStream_t s);
    static hipError_t make_ic(const PlanView<T>& pv, uint64_t seed, float* pos, float* vel, T* psi, cx<T>* work,
                              const ExecCtx& x);
    // the same path from a given white-noise field w (plain real layout)
    static hipError_t make_ic_from_noise(const PlanView<T>& pv, const T* w, float* pos, float* vel, T* psi,
                                         cx<T>* work, const ExecCtx& x);
    // d loss/d w = sum_j L_j^T g_j with g = gpsi + gpos + vfac gvel, and
    // optionally d loss/d log A = (1/2) sum g psi (one FP64 value at g_log_amp)
    static hipError_t adjoint(const PlanView<T>& pv, const T* gpsi, const float* gpos, const float* gvel,
                              const T* psi, double* g_log_amp, T* gw, cx<T>* work, hipStream_t s);
    // Eq. (1) alone: the density field delta (plain real layout) from the noise
    // of seed, or from w if not null
    static hipError_t density(const PlanView<T>& pv, uint64_t seed, const T* w, T* delta, cx<T>* work,
                              hipStream_t s);
    // binned power spectrum of a real field (pk, kmean, counts: nbins doubles);
    // the transform and the partial sums live in work
    static hipError_t power_spectrum(const PlanView<T>& pv, const T* field, int nbins, double* pk, double* kmean,
                                     double* counts, cx<T>* work, size_t work_bytes, hipStream_t s);
    // out[0..3] = mean, standard deviation, min, max of count values
    static hipError_t field_stats(const T* field, uint64_t count, double* out, double* scratch, int nblocks,
                                  hipStream_t s);
    // white-noise refinement (App. A), variant gg_refine value: parent
    // (n_parent)^3 -> child (n_parent / NL * NH)^3
    // the parent cells origin + [0, count) per axis (periodic in n_parent^3)
    static hipError_t refine(int variant, const T* parent, int n_parent, const int origin[3], int count,
                             uint64_t seed, uint32_t stream_id, T* child, hipStream_t s);
    // dst (3 fields of n_dst^3) += cloud-in-cell interpolation of the periodic
    // src (3 fields of n_src^3) at origin + m num / den (src cells)
    static hipError_t cic_add(const T* src, int n_src, int num, int den, const int origin[3], T* dst, int n_dst,
                              hipStream_t s);
    // cic_add onto the lattice of pv (n_dst = pv.n) and Eq. (3) of the result
    // at pv's lattice (origin, wrap) in the same pass
    static hipError_t cic_add_zel(const T* src, int n_src, int num, int den, const int origin[3], T* dst,
                                  const PlanView<T>& pv, float* pos, float* vel, hipStream_t s);
    // Eq. 5 on a real field: modes with n^2 >= n2_max dropped, optional CiC
    // deconvolution; out (R) may equal field; work: two plain half spectra
    // Eq. 5 as the filter of a noise field restricted to n^2 < n2_max (with
    // the cloud-in-cell deconvolution if set): psi (3 R).  The half spectrum
    // is pruned to the window's columns (work: 3 N N kc complex values); a
    // window too wide for that runs the fused path with the window.
    static hipError_t windowed_displacements(const PlanView<T>& pv, const T* w, int n2_max, int deconv, T* psi,
                                             cx<T>* work, const ExecCtx& x);
    // Eq. 5 on three fields at once (field, out: 3 consecutive R arrays, out
    // distinct from field): modes beyond the window are never transformed
    // along axes 1 and 0 (the half spectrum is pruned to the window's
    // columns).  work: 3 N N kc complex values at most (kc <= N / 2).
    static hipError_t lowpass3(const PlanView<T>& pv, const T* field, int n2_max, int deconv, T* out, cx<T>* work,
                               hipStream_t s);
    static hipError_t lowpass(const PlanView<T>& pv, const T* field, int n2_max, int deconv, T* out, cx<T>* work,
                              hipStream_t s);
    // Sec. 2.3 degrade: NGP values of the (factor n)^3 fine field on the plan's
    // lattice, moved by shift[j] coarse cells along axis j in Fourier space
    static hipError_t degrade(const PlanView<T>& pv, const T* fine, int factor, const double shift[3], T* out,
                              cx<T>* work, hipStream_t s);
    static hipError_t fused_forward(const PlanView<T>& pv, const T* w, uint64_t seed, float* pos, float* vel, T* psi,
                                    cx<T>* work, const ExecCtx& x);
    // chunk count the fused path can use for lattice n (1 = no pipelining)
    static int max_chunks(int n);
    // the tile choices of ExecCtx for lattice n: full and half line counts of
    // the axis-2 passes, and the built-in choices of the first and last pass
    static void tile_options(int n, int& full, int& half, int& p1_default, int& z_default);
    // exact table tau[ntau]; for float plans also the piecewise-cubic
    // segments (kTauSeg float4) the fused passes evaluate
    static hipError_t tau_table(T* tau, int64_t ntau, void* tauseg, int n, double box, double amp_growth2,
                                double gamma, double n_s, hipStream_t s);
    // bytes of the fused path's workspace (three half spectra without the
    // k2 = N/2 plane) and of the inverse transform's scratch (one full half
    // spectrum)
    static size_t fused_work_bytes(int n) { return 3 * (size_t)n * n * (n / 2) * sizeof(cx<T>); }
    static size_t inverse_work_bytes(int n) { return (size_t)n * n * (n / 2 + 1) * sizeof(cx<T>); }
};

// Bytes of the static workspace behind gg_make_ic_noalloc (per device).
constexpr size_t kNoallocScratchBytes = (size_t)48 << 20;

// (N_L, N_H) of a refinement variant, or (0, 0) if unknown
void refine_sizes(int variant, int& nl, int& nh);

// out[0] = scale * sum of part[0..count) in a fixed order (one work-group).
hipError_t launch_dot_final(const double* part, uint32_t count, double scale, double* out, hipStream_t s);

// Launches the FP64 sigma_8 integral (one work-group) on stream s.
hipError_t launch_sigma_integral(double lnk_min, double lnk_max, double gamma, double n_s, double radius,
                                 double* out, hipStream_t s);

}  // namespace gg
