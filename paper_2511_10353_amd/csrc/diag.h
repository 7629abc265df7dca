// Diagnostics of a field: binned power spectrum of its half spectrum and
// summary statistics.  The paper's pipeline can write the density field and
// its power spectrum beside the velocity fields (Sec. 2.1, list of outputs).
//
// Power spectrum: every stored mode n != 0 of the plain half spectrum (rows
// (k0, k1), k2 in [0, N/2]) with b = floor(|n|) < nbins adds w |F|^2, w |n|
// and w to bin b, w = 1 on the planes k2 = 0 and k2 = N/2 and 2 between them
// (the conjugate half is implied).  Then P_b = (L^3/N^6) sum w |F|^2 / sum w,
// kmean_b = k_f sum w |n| / sum w, count_b = sum w.  All sums in binary64 and
// in a fixed order: within a row the bins are contiguous runs of k2 (|n|
// grows with k2), so the first thread of each run adds the run into the
// work-group's accumulator for that bin (one writer per bin per step); rows
// follow each other in order; the work-groups' partial sums are added in
// index order by k_pk_final.  Results do not depend on scheduling.
//
// Statistics: mean, then sum (f - mean)^2, min and max, each with per-block
// partials in a fixed order and one final combining pass.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.h"

namespace gg {

constexpr int kPkThreads = 256;
constexpr int kPkMaxBins = 1024;

template <typename T>
__global__ __launch_bounds__(kPkThreads) void k_pk_rows(const cx<T>* __restrict__ spec, int n, int nbins,
                                                        int rows_per_block, double* __restrict__ part) {
    extern __shared__ double sh[];
    double* ap = sh;
    double* ak = sh + nbins;
    double* aw = sh + 2 * nbins;
    double* vp = sh + 3 * nbins;
    double* vk = vp + kPkThreads;
    double* vw = vk + kPkThreads;
    int* vb = reinterpret_cast<int*>(vw + kPkThreads);
    const int t = threadIdx.x;
    for (int i = t; i < 3 * nbins; i += kPkThreads) sh[i] = 0.0;
    const int K = n / 2 + 1;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    for (int rr = 0; rr < rows_per_block; ++rr) {
        const int64_t r = r0 + rr;
        const int k0 = (int)(r / n), k1 = (int)(r % n);
        const int s0 = k0 <= n / 2 ? k0 : k0 - n;
        const int s1 = k1 <= n / 2 ? k1 : k1 - n;
        const int c = s0 * s0 + s1 * s1;
        for (int base = 0; base < K; base += kPkThreads) {
            const int k2 = base + t;
            int b = -1;
            double p = 0.0, kk = 0.0, w = 0.0;
            if (k2 < K) {
                const int n2 = c + k2 * k2;
                int q = (int)sqrt((double)n2);
                while (q * q > n2) --q;
                while ((q + 1) * (q + 1) <= n2) ++q;
                if (n2 > 0 && q < nbins) {
                    const cx<T> f = spec[r * K + k2];
                    w = (k2 == 0 || k2 == n / 2) ? 1.0 : 2.0;
                    p = w * ((double)f.x * (double)f.x + (double)f.y * (double)f.y);
                    kk = w * sqrt((double)n2);
                    b = q;
                }
            }
            __syncthreads();  // the previous step's run sums are done with v*
            vb[t] = b;
            vp[t] = p;
            vk[t] = kk;
            vw[t] = w;
            __syncthreads();
            if (b >= 0 && (t == 0 || vb[t - 1] != b)) {
                double sp = 0.0, sk = 0.0, sw = 0.0;
                for (int u = t; u < kPkThreads && vb[u] == b; ++u) {
                    sp += vp[u];
                    sk += vk[u];
                    sw += vw[u];
                }
                ap[b] += sp;
                ak[b] += sk;
                aw[b] += sw;
            }
        }
    }
    __syncthreads();
    for (int i = t; i < 3 * nbins; i += kPkThreads) part[(int64_t)blockIdx.x * 3 * nbins + i] = sh[i];
}

template <typename T>  // T: the plan's type (one instantiation per translation unit)
__global__ void k_pk_final(const double* __restrict__ part, int nblocks, int nbins, double pscale, double kf,
                           double* __restrict__ pk, double* __restrict__ kmean, double* __restrict__ counts) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    double sp = 0.0, sk = 0.0, sw = 0.0;
    for (int g = 0; g < nblocks; ++g) {
        const double* q = part + (int64_t)g * 3 * nbins;
        sp += q[b];
        sk += q[nbins + b];
        sw += q[2 * nbins + b];
    }
    counts[b] = sw;
    pk[b] = sw > 0.0 ? sp / sw * pscale : 0.0;
    kmean[b] = sw > 0.0 ? sk / sw * kf : 0.0;
}

constexpr int kStatThreads = 256;

// part[g] = sum of the values of block g's stride (mean pass), or, with a
// mean, part[3 g .. 3 g + 2] = (sum (f - mean)^2, min, max)
template <typename T, bool SECOND>
__global__ __launch_bounds__(kStatThreads) void k_stats_partial(const T* __restrict__ f, uint64_t count,
                                                                const double* __restrict__ mean,
                                                                double* __restrict__ part) {
    __shared__ double s0[kStatThreads], s1[kStatThreads], s2[kStatThreads];
    const int t = threadIdx.x;
    const double m = SECOND ? mean[0] : 0.0;
    double a = 0.0, lo = INFINITY, hi = -INFINITY;
    for (uint64_t i = (uint64_t)blockIdx.x * kStatThreads + t; i < count; i += (uint64_t)gridDim.x * kStatThreads) {
        const double x = (double)f[i];
        if (SECOND) {
            const double d = x - m;
            a += d * d;
            lo = fmin(lo, x);
            hi = fmax(hi, x);
        } else {
            a += x;
        }
    }
    s0[t] = a;
    s1[t] = lo;
    s2[t] = hi;
    __syncthreads();
    for (int h = kStatThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            s0[t] += s0[t + h];
            s1[t] = fmin(s1[t], s1[t + h]);
            s2[t] = fmax(s2[t], s2[t + h]);
        }
        __syncthreads();
    }
    if (t == 0) {
        if (SECOND) {
            part[3 * blockIdx.x] = s0[0];
            part[3 * blockIdx.x + 1] = s1[0];
            part[3 * blockIdx.x + 2] = s2[0];
        } else {
            part[blockIdx.x] = s0[0];
        }
    }
}

// one thread: out[0] = mean (first pass) or out[1..3] = (std, min, max)
template <typename T, bool SECOND>
__global__ void k_stats_final(const double* __restrict__ part, int nblocks, uint64_t count, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (!SECOND) {
        double a = 0.0;
        for (int g = 0; g < nblocks; ++g) a += part[g];
        out[0] = a / (double)count;
    } else {
        double a = 0.0, lo = INFINITY, hi = -INFINITY;
        for (int g = 0; g < nblocks; ++g) {
            a += part[3 * g];
            lo = fmin(lo, part[3 * g + 1]);
            hi = fmax(hi, part[3 * g + 2]);
        }
        out[1] = sqrt(a / (double)count);
        out[2] = lo;
        out[3] = hi;
    }
}

}  // namespace gg
