// Batched in-LDS Stockham FFT building blocks for gfx950 (wave64).
//
// A work-group transforms L independent lines of M complex points.  Lines
// are the columns of an LDS tile of M rows x L columns; element (row, col)
// lives at row * L + (col ^ (row & (L - 1))).  L complex values of one row
// span 128 bytes (L = 16 for float, 8 for double), so every access in which
// each aligned group of L lanes touches one row (the c-fastest thread
// mapping used by all butterfly stages) or one column over L consecutive
// rows (the contiguous copies of the z passes) hits every LDS bank once.
//
// Thread t of the group works on line c = t % L as the j = t / L-th of
// TPL = M / V threads of that line; it holds V complex values in registers
// (V a multiple of every radix of the line's plan).  A stage of radix R with sub-length NS (product of the radices
// already applied) performs, for butterfly b in [0, M/R), k = b mod NS:
//   a_r = x[b + r M/R] * W_{NS R}^{r k},  A = DFT_R(a),
//   y[(b - k) R + k + r NS] = A_r,
// which leaves the result in natural order after the last stage (Stockham
// autosort).  The first stage takes its inputs from registers and the last
// stage leaves its outputs in registers, so a strided pass moves data between
// HBM and registers directly and uses LDS only for the exchanges in between.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gg {

template <typename T>
struct cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> w) { return {a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x}; }
// a * conj(w)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> w) { return {a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y}; }
// a * i
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }
// a * (DIR i): DIR = -1 is a quarter turn of the forward transform
template <int DIR, typename T>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
    if constexpr (DIR < 0) return {a.y, -a.x};
    else return {-a.y, a.x};
}
// a * W where W = (wr, DIR * wi) with compile-time constants
template <int DIR, typename T>
__device__ __forceinline__ cx<T> cmul_dir(cx<T> a, T wr, T wi) {
    const T s = (DIR < 0) ? -wi : wi;
    return {a.x * wr - a.y * s, a.x * s + a.y * wr};
}

// ---------------------------------------------------------------------------
// Small DFTs in registers: X_k = sum_n a_n exp(DIR 2 pi i n k / R).
// ---------------------------------------------------------------------------
constexpr double kSqrtHalf = 0.70710678118654752440;
constexpr double kCos8 = 0.92387953251128675613;  // cos(pi/8)
constexpr double kSin8 = 0.38268343236508977173;  // sin(pi/8)

template <int DIR, typename T>
__device__ __forceinline__ void dft2(cx<T>& a0, cx<T>& a1) {
    cx<T> t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
    cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2);
    cx<T> t2 = cadd(a1, a3), t3 = rot90<DIR>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cx<T>* a) {
    const T h = (T)kSqrtHalf;
    dft4<DIR>(a[0], a[2], a[4], a[6]);
    dft4<DIR>(a[1], a[3], a[5], a[7]);
    cx<T> o1 = cmul_dir<DIR>(a[3], h, h);
    cx<T> o2 = rot90<DIR>(a[5]);
    cx<T> o3 = cmul_dir<DIR>(a[7], -h, h);
    cx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
    a[0] = cadd(e0, o0);
    a[4] = csub(e0, o0);
    a[1] = cadd(e1, o1);
    a[5] = csub(e1, o1);
    a[2] = cadd(e2, o2);
    a[6] = csub(e2, o2);
    a[3] = cadd(e3, o3);
    a[7] = csub(e3, o3);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft16(cx<T>* a) {
    // n = 4 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle W16^(n2 k1), DFT4 over n2
    const T h = (T)kSqrtHalf, c8 = (T)kCos8, s8 = (T)kSin8;
    dft4<DIR>(a[0], a[4], a[8], a[12]);
    dft4<DIR>(a[1], a[5], a[9], a[13]);
    dft4<DIR>(a[2], a[6], a[10], a[14]);
    dft4<DIR>(a[3], a[7], a[11], a[15]);
    // a[4 k1 + n2] now holds Y[n2][k1]
    a[5] = cmul_dir<DIR>(a[5], c8, s8);     // n2=1,k1=1: W^1
    a[6] = cmul_dir<DIR>(a[6], h, h);       // n2=2,k1=1: W^2
    a[7] = cmul_dir<DIR>(a[7], s8, c8);     // n2=3,k1=1: W^3
    a[9] = cmul_dir<DIR>(a[9], h, h);       // n2=1,k1=2: W^2
    a[10] = rot90<DIR>(a[10]);              // n2=2,k1=2: W^4
    a[11] = cmul_dir<DIR>(a[11], -h, h);    // n2=3,k1=2: W^6
    a[13] = cmul_dir<DIR>(a[13], s8, c8);   // n2=1,k1=3: W^3
    a[14] = cmul_dir<DIR>(a[14], -h, h);    // n2=2,k1=3: W^6
    a[15] = cmul_dir<DIR>(a[15], -c8, -s8); // n2=3,k1=3: W^9
    dft4<DIR>(a[0], a[1], a[2], a[3]);
    dft4<DIR>(a[4], a[5], a[6], a[7]);
    dft4<DIR>(a[8], a[9], a[10], a[11]);
    dft4<DIR>(a[12], a[13], a[14], a[15]);
    // a[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4x4 index
    cx<T> t;
#define GG_SWAP(p, q) t = a[p]; a[p] = a[q]; a[q] = t;
    GG_SWAP(1, 4) GG_SWAP(2, 8) GG_SWAP(3, 12) GG_SWAP(6, 9) GG_SWAP(7, 13) GG_SWAP(11, 14)
#undef GG_SWAP
}

// radix 3: w = exp(DIR 2 pi i / 3) = -1/2 + DIR i sqrt(3)/2
constexpr double kSqrt3Half = 0.86602540378443864676;

template <int DIR, typename T>
__device__ __forceinline__ void dft3(cx<T>* a) {
    const cx<T> t = cadd(a[1], a[2]);
    const cx<T> d = cscale(rot90<DIR>(csub(a[1], a[2])), (T)kSqrt3Half);
    const cx<T> m = csub(a[0], cscale(t, (T)0.5));
    a[0] = cadd(a[0], t);
    a[1] = cadd(m, d);
    a[2] = csub(m, d);
}

// radix 5: c1 = cos(2 pi/5), c2 = cos(4 pi/5), s1 = sin(2 pi/5), s2 = sin(4 pi/5)
constexpr double kC51 = 0.30901699437494742410;
constexpr double kC52 = -0.80901699437494742410;
constexpr double kS51 = 0.95105651629515357212;
constexpr double kS52 = 0.58778525229247312917;

template <int DIR, typename T>
__device__ __forceinline__ void dft5(cx<T>* a) {
    const cx<T> t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
    const cx<T> d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
    const cx<T> m1 = cadd(a[0], cadd(cscale(t1, (T)kC51), cscale(t2, (T)kC52)));
    const cx<T> m2 = cadd(a[0], cadd(cscale(t1, (T)kC52), cscale(t2, (T)kC51)));
    const cx<T> r1 = rot90<DIR>(cadd(cscale(d1, (T)kS51), cscale(d2, (T)kS52)));
    const cx<T> r2 = rot90<DIR>(csub(cscale(d1, (T)kS52), cscale(d2, (T)kS51)));
    a[0] = cadd(a[0], cadd(t1, t2));
    a[1] = cadd(m1, r1);
    a[4] = csub(m1, r1);
    a[2] = cadd(m2, r2);
    a[3] = csub(m2, r2);
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* a) {
    if constexpr (R == 2) dft2<DIR>(a[0], a[1]);
    else if constexpr (R == 3) dft3<DIR>(a);
    else if constexpr (R == 4) dft4<DIR>(a[0], a[1], a[2], a[3]);
    else if constexpr (R == 5) dft5<DIR>(a);
    else if constexpr (R == 8) dft8<DIR>(a);
    else if constexpr (R == 16) dft16<DIR>(a);
    else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// Radix plans: line length M -> radices of the forward transform (the inverse
// applies them in reverse order so that its first stage reads the positions
// the forward's last stage leaves in registers).
// ---------------------------------------------------------------------------
// V: complex values per thread (every radix of the plan divides it); a
// thread performs V / R butterflies of each radix-R stage.  The mixed-radix
// plans serve the uneven lattices (N = 96, 160, 192 and their r2c halves).
template <int M> struct Plan;
template <> struct Plan<4>    { static constexpr int S = 1, V = 4;  static constexpr int R[1] = {4}; };
template <> struct Plan<8>    { static constexpr int S = 1, V = 8;  static constexpr int R[1] = {8}; };
template <> struct Plan<16>   { static constexpr int S = 1, V = 16; static constexpr int R[1] = {16}; };
template <> struct Plan<32>   { static constexpr int S = 2, V = 8;  static constexpr int R[2] = {8, 4}; };
template <> struct Plan<48>   { static constexpr int S = 3, V = 12; static constexpr int R[3] = {4, 4, 3}; };
template <> struct Plan<64>   { static constexpr int S = 2, V = 8;  static constexpr int R[2] = {8, 8}; };
template <> struct Plan<80>   { static constexpr int S = 3, V = 20; static constexpr int R[3] = {4, 4, 5}; };
template <> struct Plan<96>   { static constexpr int S = 3, V = 24; static constexpr int R[3] = {8, 4, 3}; };
template <> struct Plan<128>  { static constexpr int S = 2, V = 16; static constexpr int R[2] = {16, 8}; };
template <> struct Plan<160>  { static constexpr int S = 4, V = 20; static constexpr int R[4] = {4, 4, 2, 5}; };
template <> struct Plan<192>  { static constexpr int S = 3, V = 24; static constexpr int R[3] = {8, 8, 3}; };
template <> struct Plan<256>  { static constexpr int S = 2, V = 16; static constexpr int R[2] = {16, 16}; };
template <> struct Plan<512>  { static constexpr int S = 3, V = 8;  static constexpr int R[3] = {8, 8, 8}; };
template <> struct Plan<1024> { static constexpr int S = 3, V = 16; static constexpr int R[3] = {16, 4, 16}; };

template <int M>
struct PlanInfo {
    static constexpr bool valid() {
        int prod = 1;
        for (int s = 0; s < Plan<M>::S; ++s) {
            if (Plan<M>::V % Plan<M>::R[s] != 0) return false;
            prod *= Plan<M>::R[s];
        }
        return prod == M && M % Plan<M>::V == 0;
    }
    static_assert(valid(), "radices must multiply to M and divide V");
    static constexpr int V = Plan<M>::V;   // complex values held per thread
    static constexpr int RMAX = V;
    static constexpr int TPL = M / V;      // threads per line
    template <int DIR>
    static constexpr int first_radix() { return DIR < 0 ? Plan<M>::R[0] : Plan<M>::R[Plan<M>::S - 1]; }
    template <int DIR>
    static constexpr int last_radix() { return DIR < 0 ? Plan<M>::R[Plan<M>::S - 1] : Plan<M>::R[0]; }
};

// Position (row) of register slot i of thread j before the first stage ...
template <int M, int DIR>
__device__ __forceinline__ int first_pos(int j, int i) {
    constexpr int R = PlanInfo<M>::template first_radix<DIR>();
    return j + PlanInfo<M>::TPL * (i / R) + (i % R) * (M / R);
}
// ... and after the last stage.
template <int M, int DIR>
__device__ __forceinline__ int last_pos(int j, int i) {
    constexpr int R = PlanInfo<M>::template last_radix<DIR>();
    return j + PlanInfo<M>::TPL * (i / R) + (i % R) * (M / R);
}

template <int L>
__device__ __forceinline__ int lidx(int row, int col) { return row * L + (col ^ (row & (L - 1))); }

// The 1024-point plan (16, 4, 16) with 64 threads per line: the exchange
// between the radix-4 stage and the last radix-16 stage sends the outputs of
// thread j only to the threads j % 16 + 16 r, r < 4.  Placing thread j of a
// line in 16-lane row j / 16 of a wave (float tiles, 16 lines: wave j % 16,
// lane 16 (j / 16) + column; double tiles, 8 lines: wave (j % 16) / 2, lane
// 16 (j / 16) + 8 (j % 2) + column) puts those four threads in the four rows
// of one wave at the same position within the row, so the exchange is a 4 x 4
// transpose across rows, two lane swaps per 32-bit register
// (v_permlane32_swap, then v_permlane16_swap), instead of an LDS round trip
// and a work-group barrier.
template <typename T, int M, int L>
struct RowExchange {
    static constexpr bool value = M == 1024 && PlanInfo<M>::TPL == 64 && Plan<M>::S == 3 && Plan<M>::R[0] == 16 &&
                                  Plan<M>::R[1] == 4 && Plan<M>::R[2] == 16 &&
                                  ((sizeof(T) == 4 && L == 16) || (sizeof(T) == 8 && L == 8));
};

// Line-local thread index j of work-group thread t (the column is t % L);
// RX: the row-exchange placement above.
template <bool RX, int L>
__device__ __forceinline__ int line_thread(int t) {
    if constexpr (RX && L == 16) return (t >> 6) + 16 * ((t & 63) >> 4);
    else if constexpr (RX && L == 8) return 2 * (t >> 6) + ((t >> 3) & 1) + 16 * ((t & 63) >> 4);
    else return t / L;
}

// x_r <- x of row r (16-lane rows of the wave) held in the caller's register
// q = own row: a 4 x 4 transpose of four registers across the four rows.
__device__ __forceinline__ void row_transpose4(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3) {
    const auto a = __builtin_amdgcn_permlane32_swap(x0, x2, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(x1, x3, false, false);
    const auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
    const auto d = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
    x0 = c[0];
    x1 = c[1];
    x2 = d[0];
    x3 = d[1];
}

// One Stockham stage (see the file header).  tw[m * TWS] = exp(-2 pi i m / M).
// RIN: the stage's inputs are already in registers (after a row exchange);
// ROUT: the outputs go to the next stage by the row exchange, not LDS.
template <typename T, int M, int L, int R, int NS, int DIR, int TWS, bool FIRST, bool LAST, bool RIN = false,
          bool ROUT = false>
__device__ __forceinline__ void stockham_stage(cx<T>* v, cx<T>* lds, const cx<T>* __restrict__ tw, int c, int j) {
    constexpr int TPL = PlanInfo<M>::TPL;
    constexpr int BPT = PlanInfo<M>::RMAX / R;
    constexpr int NB = M / R;
    if constexpr (!FIRST && !RIN) {
#pragma unroll
        for (int u = 0; u < BPT; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r) v[u * R + r] = lds[lidx<L>(j + TPL * u + r * NB, c)];
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int b = j + TPL * u;
        const int k = (int)((unsigned)b % (unsigned)NS);
        if constexpr (!FIRST) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cx<T> w = tw[(r * k * (M / (NS * R))) * TWS];
                v[u * R + r] = (DIR < 0) ? cmul(v[u * R + r], w) : cmulc(v[u * R + r], w);
            }
        }
        dft<R, DIR>(v + u * R);
        if constexpr (ROUT) {
            // output r of this thread's butterfly u goes to row r of the wave, slot
            // 4 u + (own row): transpose the four outputs across the rows
            static_assert(R == 4, "row exchange is a 4 x 4 transpose");
            constexpr int W = sizeof(T) / 4;  // 32-bit words per component
            uint32_t re[W][4], im[W][4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                __builtin_memcpy(&re[0][r], &v[u * R + r].x, 4);
                __builtin_memcpy(&im[0][r], &v[u * R + r].y, 4);
                if constexpr (W == 2) {
                    __builtin_memcpy(&re[1][r], reinterpret_cast<const char*>(&v[u * R + r].x) + 4, 4);
                    __builtin_memcpy(&im[1][r], reinterpret_cast<const char*>(&v[u * R + r].y) + 4, 4);
                }
            }
#pragma unroll
            for (int h = 0; h < W; ++h) {
                row_transpose4(re[h][0], re[h][1], re[h][2], re[h][3]);
                row_transpose4(im[h][0], im[h][1], im[h][2], im[h][3]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                __builtin_memcpy(&v[u * R + r].x, &re[0][r], 4);
                __builtin_memcpy(&v[u * R + r].y, &im[0][r], 4);
                if constexpr (W == 2) {
                    __builtin_memcpy(reinterpret_cast<char*>(&v[u * R + r].x) + 4, &re[1][r], 4);
                    __builtin_memcpy(reinterpret_cast<char*>(&v[u * R + r].y) + 4, &im[1][r], 4);
                }
            }
        } else if constexpr (!LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lidx<L>((b - k) * R + k + r * NS, c)] = v[u * R + r];
        }
    }
    if constexpr (!LAST && !ROUT) __syncthreads();
}

// Full transform of one line per column: inputs in v at first_pos, outputs
// in v at last_pos.  On return every thread has finished with LDS.  RX: the
// exchange before the last stage runs across the rows of each wave (threads
// placed by line_thread<true>); only for plans with RowExchange.
template <typename T, int M, int L, int DIR, int TWS, bool RX = false, int s = 0, int NS = 1>
__device__ __forceinline__ void fft_lines(cx<T>* v, cx<T>* lds, const cx<T>* __restrict__ tw, int c, int j) {
    static_assert(!RX || RowExchange<T, M, L>::value, "row exchange needs the (16, 4, 16) float plan");
    constexpr int S = Plan<M>::S;
    constexpr int R = (DIR < 0) ? Plan<M>::R[s] : Plan<M>::R[S - 1 - s];
    stockham_stage<T, M, L, R, NS, DIR, TWS, (s == 0), (s == S - 1), RX && s == 2, RX && s == 1>(v, lds, tw, c, j);
    if constexpr (s + 1 < S) fft_lines<T, M, L, DIR, TWS, RX, s + 1, NS * R>(v, lds, tw, c, j);
}

// Lines per work-group: one 128-byte LDS row of complex values.
template <typename T>
struct Tile {
    static constexpr int L = 128 / (2 * sizeof(T));
};

}  // namespace gg
