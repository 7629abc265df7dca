// C ABI of the initial-conditions library (declared in include/gg.h):
// argument validation, plan construction (FP64 twiddles, the GPU sigma_8
// integral and the tau table) and dispatch to the per-type launchers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "gg.h"
#include "diag.h"
#include "kernels.h"
#include "refine.h"
#include "ops.h"

namespace {

thread_local std::string g_last_error;

gg_status fail(gg_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

gg_status fail_hip(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return GG_ERR_HIP;
}

constexpr int kTimingSlots = 64;
constexpr int kMaxDegrade = 16;     // largest resolution-degrade factor   // calls recorded per gg_timing_read
constexpr int kPasses = 5;
constexpr int kMaxChunks = 8;
constexpr int kLaunchesMax = 4 * kMaxChunks + 1;  // launches of one gg_make_ic

}  // namespace

struct gg_plan {
    int n = 0;
    double box = 0;
    gg_dtype dtype = GG_F32;
    gg_cosmo cosmo{};
    int device = 0;
    void* tw = nullptr;    // N complex values of the dtype
    void* tau = nullptr;   // ntau values of the dtype
    int64_t ntau = 0;
    // piecewise tau: kTauSeg float4 followed by the noise's logarithm table
    // (kLnTab double2) for float plans, kTauSeg64 x 8 doubles for double plans
    void* tauseg = nullptr;
    double amplitude = 0, sigma_int = 0, growth = 0, vfac = 0, cell = 0;
    // tile choices of the fused path (0 = built-in; set by gg_plan_set_tuning
    // or gg_plan_autotune)
    int p1_lines = 0, z_lines = 0;
    // compute units of the plan's device (grids of the persistent passes)
    int cus = 0;
    // pipelined launch of the fused path: auxiliary stream, dependency events
    int nchunk = 1;
    hipStream_t aux = nullptr;
    std::vector<hipEvent_t> sync;  // 2 kMaxChunks + 3
    // timing records
    bool timing = false;
    std::vector<hipEvent_t> events;  // kTimingSlots * 2 * kLaunchesMax
    int recorded = 0;
};

namespace {

bool aligned(const void* p) { return ((uintptr_t)p & 255u) == 0; }

// The integer a caller passed for an enum parameter.  A C caller may pass any
// int; in C++ reading an enum object that holds a value outside the
// enumeration's range is undefined, so validation reads the representation.
template <typename E>
int32_t enum_bits(const E& e) {
    static_assert(sizeof(E) == sizeof(int32_t), "enums of the ABI are int-sized");
    int32_t v;
    std::memcpy(&v, &e, sizeof v);
    return v;
}

bool valid_dtype(const gg_dtype& d) {
    const int32_t v = enum_bits(d);
    return v == GG_F32 || v == GG_F64;
}

// Workspace of gg_make_ic_noalloc: one static array per device, found once
// per device (gg_plan_create, with the plan's device current) through
// hipGetSymbolAddress.  Host code uses only the recorded device address;
// the array's own name is a host-side stand-in that no kernel may receive.
constexpr size_t kScratchBytes = gg::kNoallocScratchBytes;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

gg_status scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(GG_ERR_INTERNAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return GG_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail_hip(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = ptr;
    return GG_OK;
}

void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

// launch context of the fused path for plan p on the caller's stream
gg::ExecCtx fused_ctx(gg_plan* p, void* stream) {
    gg::ExecCtx x;
    x.a = static_cast<hipStream_t>(stream);
    x.b = p->aux;
    x.sync = p->sync.empty() ? nullptr : p->sync.data();
    x.nchunk = p->nchunk;
    x.p1_lines = p->p1_lines;
    x.z_lines = p->z_lines;
    x.cus = p->cus;
    return x;
}

// Test hook: GG_FAULT_INJECT names one failure to simulate ("plan_alloc": the
// last device allocation of gg_plan_create fails; "launch": gg_make_ic
// reports a failed launch without launching).  Unset, it changes nothing.
bool fault_injected(const char* point) {
    const char* v = std::getenv("GG_FAULT_INJECT");
    return v && std::strcmp(v, point) == 0;
}

template <typename T>
gg::PlanView<T> view(const gg_plan* p) {
    gg::PlanView<T> v;
    v.n = p->n;
    v.box = p->box;
    v.cell = p->cell;
    v.offset = p->cosmo.lattice_offset;
    v.vfac = p->vfac;
    v.tw = static_cast<const gg::cx<T>*>(p->tw);
    v.tau = static_cast<const T*>(p->tau);
    v.tauseg = std::is_same_v<T, float> ? static_cast<const float4*>(p->tauseg) : nullptr;
    v.tauseg64 = std::is_same_v<T, double> ? static_cast<const double2*>(p->tauseg) : nullptr;
    v.lntab = std::is_same_v<T, float> ? reinterpret_cast<const double2*>(static_cast<const char*>(p->tauseg) +
                                                                       gg::kTauSeg * sizeof(float4))
                                       : nullptr;
    v.amp_scale = 1.0;
    v.n2_lo = 0;
    v.n2_hi = 0x7FFFFFFF;
    v.deconv = 0;
    v.origin[0] = v.origin[1] = v.origin[2] = 0.0;
    v.wrap = p->box;
    return v;
}

size_t elem_size(gg_dtype d) { return d == GG_F64 ? sizeof(double) : sizeof(float); }

gg_status check_device(const gg_plan* p) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev != p->device) return fail(GG_ERR_INVALID_ARG, "current HIP device differs from the plan's device");
    return GG_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

// Twiddles exp(-2 pi i m / N) in extended precision, rounded to the dtype.
template <typename T>
std::vector<gg::cx<T>> make_twiddles(int n) {
    std::vector<gg::cx<T>> tw(n);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int m = 0; m < n; ++m) {
        // reduce to the first octant so that special angles come out exact
        int k = m % n;
        long double c, s;
        const int q = (4 * k) / n;           // quadrant
        const int r = 4 * k - q * n;         // 4 * angle within quadrant, in units of 2 pi / (4 n)
        const long double a = two_pi * (long double)r / (4.0L * n);
        const long double ca = cosl(a), sa = sinl(a);
        switch (q) {
            case 0: c = ca; s = sa; break;
            case 1: c = -sa; s = ca; break;
            case 2: c = -ca; s = -sa; break;
            default: c = sa; s = -ca; break;
        }
        tw[m] = {(T)(double)c, (T)(double)(-s)};
    }
    return tw;
}

}  // namespace

extern "C" {

const char* gg_status_string(gg_status st) {
    switch (st) {
        case GG_OK: return "GG_OK";
        case GG_ERR_INVALID_ARG: return "GG_ERR_INVALID_ARG";
        case GG_ERR_UNSUPPORTED_SIZE: return "GG_ERR_UNSUPPORTED_SIZE";
        case GG_ERR_OUT_OF_MEMORY: return "GG_ERR_OUT_OF_MEMORY";
        case GG_ERR_HIP: return "GG_ERR_HIP";
        case GG_ERR_INTERNAL: return "GG_ERR_INTERNAL";
    }
    return "GG_ERR_UNKNOWN";
}

const char* gg_last_error(void) { return g_last_error.c_str(); }

size_t gg_workspace_bytes(const gg_plan* p) {
    if (!p) return 0;
    size_t a, b;
    if (p->dtype == GG_F64) {
        a = gg::Ops<double>::fused_work_bytes(p->n);
        b = gg::Ops<double>::inverse_work_bytes(p->n);
    } else {
        a = gg::Ops<float>::fused_work_bytes(p->n);
        b = gg::Ops<float>::inverse_work_bytes(p->n);
    }
    return a > b ? a : b;
}

gg_status gg_plan_create(gg_plan** out, const gg_grid* grid, const gg_cosmo* cosmo, gg_dtype dtype) {
    g_last_error.clear();
    if (!out || !grid || !cosmo) return fail(GG_ERR_INVALID_ARG, "null argument to gg_plan_create");
    if (!valid_dtype(dtype)) return fail(GG_ERR_INVALID_ARG, "dtype must be GG_F32 or GG_F64");
    if (!gg::supported_n(grid->n))
        return fail(GG_ERR_UNSUPPORTED_SIZE,
                    "N must be a power of two in [8, 1024] or one of 96, 160, 192, got " + std::to_string(grid->n));
    const gg_cosmo& c = *cosmo;
    if (!(grid->box > 0) || !std::isfinite(grid->box)) return fail(GG_ERR_INVALID_ARG, "box must be > 0");
    if (!(c.omega_m > 0 && c.omega_m <= 1)) return fail(GG_ERR_INVALID_ARG, "omega_m must be in (0, 1]");
    if (!(c.h > 0) || !std::isfinite(c.h)) return fail(GG_ERR_INVALID_ARG, "h must be > 0");
    if (!std::isfinite(c.n_s)) return fail(GG_ERR_INVALID_ARG, "n_s must be finite");
    if (!(c.z_init > -1) || !std::isfinite(c.z_init)) return fail(GG_ERR_INVALID_ARG, "z_init must be > -1");
    if (!(c.amp >= 0) || !std::isfinite(c.amp)) return fail(GG_ERR_INVALID_ARG, "amp must be >= 0");
    if (c.amp == 0 && !(c.sigma8 > 0)) return fail(GG_ERR_INVALID_ARG, "sigma8 must be > 0 when amp = 0");
    if (!(c.lattice_offset >= 0 && c.lattice_offset < 1))
        return fail(GG_ERR_INVALID_ARG, "lattice_offset must be in [0, 1) cells");

    gg_plan* p = new (std::nothrow) gg_plan();
    if (!p) return fail(GG_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->n = grid->n;
    p->box = grid->box;
    p->dtype = dtype;
    p->cosmo = c;
    p->cell = grid->box / (double)grid->n;
    hipError_t e = hipGetDevice(&p->device);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "hipGetDevice / compute unit count");
    }
    {
        const gg_status ss = scratch_setup(p->device);
        if (ss != GG_OK) {
            delete p;
            return ss;
        }
    }
    p->cus = cus > 0 ? cus : 256;
    // GG_CUS (tests): size the persistent passes' grids for fewer compute units
    if (const char* env = std::getenv("GG_CUS")) {
        const int want = std::atoi(env);
        if (want >= 1 && want < p->cus) p->cus = want;
    }
    const size_t es = elem_size(dtype);
    const int half = p->n / 2;
    p->ntau = 3LL * half * half + 1;
    double* d_sig = nullptr;
    hipStream_t s = nullptr;
    gg_status st = GG_OK;
    auto cleanup = [&]() {
        if (d_sig) (void)hipFree(d_sig);
        if (s) (void)hipStreamDestroy(s);
    };
    do {
        if ((e = hipMalloc(&p->tw, 2 * es * p->n)) != hipSuccess ||
            (e = hipMalloc(&p->tau, es * p->ntau)) != hipSuccess || (e = hipMalloc(&d_sig, sizeof(double))) != hipSuccess ||
            (e = fault_injected("plan_alloc")
                     ? hipErrorOutOfMemory
                     : hipMalloc(&p->tauseg, dtype == GG_F32 ? gg::kTauSeg * sizeof(float4) + gg::kLnTab * sizeof(double2)
                                                             : gg::kTauSeg64 * (gg::kTauDeg64 + 1) * sizeof(double))) !=
                hipSuccess) {
            st = fail(GG_ERR_OUT_OF_MEMORY, std::string("hipMalloc of plan tables: ") + hipGetErrorString(e));
            break;
        }
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) {
            st = fail_hip(e, "hipStreamCreate");
            break;
        }
        if (dtype == GG_F64) {
            auto tw = make_twiddles<double>(p->n);
            e = hipMemcpyAsync(p->tw, tw.data(), tw.size() * sizeof(tw[0]), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        } else {
            auto tw = make_twiddles<float>(p->n);
            std::array<double2, gg::kLnTab> lnt;
            gg::make_ln_table(lnt.data());
            e = hipMemcpyAsync(p->tw, tw.data(), tw.size() * sizeof(tw[0]), hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(static_cast<char*>(p->tauseg) + gg::kTauSeg * sizeof(float4), lnt.data(),
                                   sizeof(lnt), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        if (e != hipSuccess) {
            st = fail_hip(e, "twiddle upload");
            break;
        }
        const double gamma = c.omega_m * c.h;
        e = gg::launch_sigma_integral(std::log(1e-5), std::log(1e3), gamma, c.n_s, 8.0, d_sig, s);
        double sig = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&sig, d_sig, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            st = fail_hip(e, "sigma_8 integral");
            break;
        }
        if (!(sig > 0) || !std::isfinite(sig)) {
            st = fail(GG_ERR_INTERNAL, "sigma_8 integral is not positive");
            break;
        }
        p->sigma_int = sig;
        p->amplitude = c.amp > 0 ? c.amp : c.sigma8 * c.sigma8 / sig;
        p->growth = 1.0 / (1.0 + c.z_init);
        const double a = 1.0 / (1.0 + c.z_init);
        p->vfac = a * (100.0 * std::sqrt(c.omega_m / std::pow(a, 3.0) + 1.0 - c.omega_m)) * 1.0;
        const double ag2 = p->amplitude * p->growth * p->growth;
        if (dtype == GG_F64)
            e = gg::Ops<double>::tau_table(static_cast<double*>(p->tau), p->ntau, p->tauseg, p->n, p->box, ag2, gamma,
                                           c.n_s, s);
        else
            e = gg::Ops<float>::tau_table(static_cast<float*>(p->tau), p->ntau, p->tauseg, p->n, p->box, ag2, gamma,
                                          c.n_s, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            st = fail_hip(e, "tau table");
            break;
        }
        // pipelining of the fused path: GG_CHUNKS overrides the default chunk count
        int nc = dtype == GG_F64 ? gg::Ops<double>::max_chunks(p->n) : gg::Ops<float>::max_chunks(p->n);
        if (const char* env = std::getenv("GG_CHUNKS")) {
            const int want = std::atoi(env);
            const int cblocks = (p->n / 2) / (dtype == GG_F64 ? gg::Tile<double>::L : gg::Tile<float>::L);
            if (want == 1 || (want >= 1 && want <= kMaxChunks && p->n >= 256 && (p->n / 8) % want == 0 &&
                              cblocks % want == 0))
                nc = want;
        }
        p->nchunk = nc;
        if (p->n >= 256) {  // pipelining possible: stream and events for any chunk count
            if ((e = hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking)) != hipSuccess) {
                st = fail_hip(e, "hipStreamCreate (auxiliary)");
                break;
            }
            p->sync.resize(2 * kMaxChunks + 3, nullptr);
            for (auto& ev : p->sync) {
                if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) break;
            }
            if (e != hipSuccess) {
                st = fail_hip(e, "hipEventCreate (sync)");
                break;
            }
        }
    } while (false);
    cleanup();
    if (st != GG_OK) {
        for (hipEvent_t ev : p->sync)
            if (ev) (void)hipEventDestroy(ev);
        if (p->aux) (void)hipStreamDestroy(p->aux);
        if (p->tw) (void)hipFree(p->tw);
        if (p->tau) (void)hipFree(p->tau);
        if (p->tauseg) (void)hipFree(p->tauseg);
        delete p;
        return st;
    }
    *out = p;
    return GG_OK;
}

gg_status gg_plan_destroy(gg_plan* p) {
    if (!p) return GG_OK;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != p->device) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (hipEvent_t ev : p->events) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : p->sync)
        if (ev) (void)hipEventDestroy(ev);
    if (p->aux) (void)hipStreamDestroy(p->aux);
    if (p->tw) (void)hipFree(p->tw);
    if (p->tau) (void)hipFree(p->tau);
    if (p->tauseg) (void)hipFree(p->tauseg);
    if (cur >= 0 && cur != p->device) (void)hipSetDevice(cur);
    delete p;
    return GG_OK;
}

gg_status gg_plan_query(const gg_plan* p, gg_plan_info* info) {
    if (!p || !info) return fail(GG_ERR_INVALID_ARG, "null argument to gg_plan_query");
    info->n = p->n;
    info->dtype = p->dtype;
    info->box = p->box;
    info->amplitude = p->amplitude;
    info->sigma8_integral = p->sigma_int;
    info->growth = p->growth;
    info->velocity_factor = p->vfac;
    info->real_elems = (size_t)p->n * p->n * p->n;
    info->spectrum_elems = (size_t)p->n * p->n * (p->n / 2 + 1);
    info->workspace_bytes = gg_workspace_bytes(p);
    info->chunks = p->nchunk;
    {
        int full = 0, half = 0, p1d = 0, zd = 0;
        if (p->dtype == GG_F64) gg::Ops<double>::tile_options(p->n, full, half, p1d, zd);
        else gg::Ops<float>::tile_options(p->n, full, half, p1d, zd);
        info->p1_lines = p->p1_lines ? p->p1_lines : p1d;
        info->z_lines = p->z_lines ? p->z_lines : zd;
    }
    return GG_OK;
}

gg_status gg_noise(const gg_plan* p, uint64_t seed, uint32_t stream_id, void* w, void* stream) {
    if (!p || !w) return fail(GG_ERR_INVALID_ARG, "null argument to gg_noise");
    if (!aligned(w)) return fail(GG_ERR_INVALID_ARG, "w must be 256-byte aligned");
    gg_status st = check_device(p);
    if (st != GG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = p->dtype == GG_F64
                       ? gg::Ops<double>::noise(view<double>(p), seed, stream_id, static_cast<double*>(w), s)
                       : gg::Ops<float>::noise(view<float>(p), seed, stream_id, static_cast<float*>(w), s);
    return e == hipSuccess ? GG_OK : fail_hip(e, "noise launch");
}

gg_status gg_fft3d(const gg_plan* p, int dir, const void* in, void* out, void* work, void* stream) {
    if (!p || !in || !out) return fail(GG_ERR_INVALID_ARG, "null argument to gg_fft3d");
    if (dir != 1 && dir != -1) return fail(GG_ERR_INVALID_ARG, "dir must be +1 or -1");
    if (!aligned(in) || !aligned(out)) return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t es = elem_size(p->dtype);
    const size_t rbytes = es * p->n * p->n * p->n;
    const size_t hbytes = 2 * es * p->n * p->n * (p->n / 2 + 1);
    if (dir == 1 ? overlap(in, rbytes, out, hbytes) : overlap(in, hbytes, out, rbytes))
        return fail(GG_ERR_INVALID_ARG, "in and out must not overlap");
    if (dir == -1) {
        if (!work) return fail(GG_ERR_INVALID_ARG, "the inverse transform needs a work buffer");
        if (!aligned(work)) return fail(GG_ERR_INVALID_ARG, "work must be 256-byte aligned");
        if (overlap(work, hbytes, in, hbytes) || overlap(work, hbytes, out, rbytes))
            return fail(GG_ERR_INVALID_ARG, "work must not overlap in or out");
    }
    gg_status st = check_device(p);
    if (st != GG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (p->dtype == GG_F64) {
        using C = gg::cx<double>;
        e = dir == 1 ? gg::Ops<double>::fft_forward(view<double>(p), static_cast<const double*>(in), static_cast<C*>(out), s)
                     : gg::Ops<double>::fft_inverse(view<double>(p), static_cast<const C*>(in), static_cast<double*>(out),
                                                     static_cast<C*>(work), s);
    } else {
        using C = gg::cx<float>;
        e = dir == 1 ? gg::Ops<float>::fft_forward(view<float>(p), static_cast<const float*>(in), static_cast<C*>(out), s)
                     : gg::Ops<float>::fft_inverse(view<float>(p), static_cast<const C*>(in), static_cast<float*>(out),
                                                    static_cast<C*>(work), s);
    }
    return e == hipSuccess ? GG_OK : fail_hip(e, "fft3d launch");
}

gg_status gg_filter(const gg_plan* p, const void* spec_in, void* psi_spec, void* delta_spec, void* stream) {
    if (!p || !spec_in || !psi_spec) return fail(GG_ERR_INVALID_ARG, "null argument to gg_filter");
    if (!aligned(spec_in) || !aligned(psi_spec) || (delta_spec && !aligned(delta_spec)))
        return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t hbytes = 2 * elem_size(p->dtype) * p->n * p->n * (p->n / 2 + 1);
    if (overlap(spec_in, hbytes, psi_spec, 3 * hbytes) || (delta_spec && overlap(spec_in, hbytes, delta_spec, hbytes)) ||
        (delta_spec && overlap(psi_spec, 3 * hbytes, delta_spec, hbytes)))
        return fail(GG_ERR_INVALID_ARG, "filter buffers must not overlap");
    gg_status st = check_device(p);
    if (st != GG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (p->dtype == GG_F64) {
        using C = gg::cx<double>;
        e = gg::Ops<double>::filter(view<double>(p), static_cast<const C*>(spec_in), static_cast<C*>(psi_spec),
                                    static_cast<C*>(delta_spec), s);
    } else {
        using C = gg::cx<float>;
        e = gg::Ops<float>::filter(view<float>(p), static_cast<const C*>(spec_in), static_cast<C*>(psi_spec),
                                   static_cast<C*>(delta_spec), s);
    }
    return e == hipSuccess ? GG_OK : fail_hip(e, "filter launch");
}

gg_status gg_zeldovich(const gg_plan* p, const void* psi, float* pos, float* vel, void* stream) {
    if (!p || !psi || !pos || !vel) return fail(GG_ERR_INVALID_ARG, "null argument to gg_zeldovich");
    if (!aligned(psi) || !aligned(pos) || !aligned(vel))
        return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t n3 = (size_t)p->n * p->n * p->n;
    if (overlap(pos, 12 * n3, vel, 12 * n3) || overlap(psi, 3 * n3 * elem_size(p->dtype), pos, 12 * n3) ||
        overlap(psi, 3 * n3 * elem_size(p->dtype), vel, 12 * n3))
        return fail(GG_ERR_INVALID_ARG, "psi, pos and vel must not overlap");
    gg_status st = check_device(p);
    if (st != GG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = p->dtype == GG_F64
                       ? gg::Ops<double>::zeldovich(view<double>(p), static_cast<const double*>(psi), pos, vel, s)
                       : gg::Ops<float>::zeldovich(view<float>(p), static_cast<const float*>(psi), pos, vel, s);
    return e == hipSuccess ? GG_OK : fail_hip(e, "zeldovich launch");
}

gg_status gg_make_ic(const gg_plan* pc, uint64_t seed, float* pos, float* vel, void* psi_opt, void* work,
                     void* stream) {
    if (!pc || !pos || !vel || !work) return fail(GG_ERR_INVALID_ARG, "null argument to gg_make_ic");
    if (!aligned(pos) || !aligned(vel) || !aligned(work) || (psi_opt && !aligned(psi_opt)))
        return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t n3 = (size_t)pc->n * pc->n * pc->n;
    const size_t wb = gg_workspace_bytes(pc);
    const size_t pb = psi_opt ? 3 * n3 * elem_size(pc->dtype) : 0;
    if (overlap(pos, 12 * n3, vel, 12 * n3) || overlap(work, wb, pos, 12 * n3) || overlap(work, wb, vel, 12 * n3) ||
        (psi_opt && (overlap(psi_opt, pb, work, wb) || overlap(psi_opt, pb, pos, 12 * n3) ||
                     overlap(psi_opt, pb, vel, 12 * n3))))
        return fail(GG_ERR_INVALID_ARG, "pos, vel, psi and work must not overlap");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    gg_plan* p = const_cast<gg_plan*>(pc);  // timing records are the plan's only mutable state
    gg::ExecCtx x = fused_ctx(p, stream);
    if (p->timing && p->recorded < kTimingSlots) {
        x.tev = &p->events[(size_t)p->recorded * 2 * kLaunchesMax];
        p->recorded++;
    }
    hipError_t e;
    if (fault_injected("launch"))
        e = hipErrorLaunchFailure;
    else if (p->dtype == GG_F64)
        e = gg::Ops<double>::make_ic(view<double>(p), seed, pos, vel, static_cast<double*>(psi_opt),
                                     static_cast<gg::cx<double>*>(work), x);
    else
        e = gg::Ops<float>::make_ic(view<float>(p), seed, pos, vel, static_cast<float*>(psi_opt),
                                    static_cast<gg::cx<float>*>(work), x);
    return e == hipSuccess ? GG_OK : fail_hip(e, "make_ic launch");
}

gg_status gg_make_ic_noalloc(const gg_plan* pc, uint64_t seed, float* pos, float* vel, void* psi_opt, void* stream) {
    if (!pc || !pos || !vel) return fail(GG_ERR_INVALID_ARG, "null argument to gg_make_ic_noalloc");
    const size_t wb = gg_workspace_bytes(pc);
    if (wb > kScratchBytes)
        return fail(GG_ERR_UNSUPPORTED_SIZE,
                    "gg_make_ic_noalloc: this lattice needs " + std::to_string(wb) + " bytes of workspace, the static "
                    "scratch holds " + std::to_string(kScratchBytes) + " (float lattices up to 160^3, double up to "
                    "128^3); use gg_make_ic with a workspace");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    void* ws = scratch_ptr(pc->device);
    if (!ws) return fail(GG_ERR_INTERNAL, "no scratch address recorded for the plan's device");
    return gg_make_ic(pc, seed, pos, vel, psi_opt, ws, stream);
}

gg_status gg_make_ic_from_noise(const gg_plan* pc, const void* w, double amp_scale, float* pos, float* vel,
                                void* psi_opt, void* work, void* stream) {
    if (!pc || !w || !work) return fail(GG_ERR_INVALID_ARG, "null argument to gg_make_ic_from_noise");
    if (!pos != !vel) return fail(GG_ERR_INVALID_ARG, "pos and vel must both be given or both be NULL");
    if (!pos && !psi_opt) return fail(GG_ERR_INVALID_ARG, "nothing to write: give pos/vel or psi");
    if (!(amp_scale > 0) || !std::isfinite(amp_scale)) return fail(GG_ERR_INVALID_ARG, "amp_scale must be > 0");
    if (!aligned(w) || !aligned(work) || (pos && (!aligned(pos) || !aligned(vel))) || (psi_opt && !aligned(psi_opt)))
        return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t n3 = (size_t)pc->n * pc->n * pc->n;
    const size_t es = elem_size(pc->dtype);
    const size_t wb = gg_workspace_bytes(pc);
    if (overlap(w, es * n3, work, wb) || (psi_opt && (overlap(psi_opt, 3 * es * n3, work, wb) ||
                                                      overlap(psi_opt, 3 * es * n3, w, es * n3))) ||
        (pos && (overlap(pos, 12 * n3, vel, 12 * n3) || overlap(pos, 12 * n3, work, wb) ||
                 overlap(vel, 12 * n3, work, wb))))
        return fail(GG_ERR_INVALID_ARG, "w, pos, vel, psi and work must not overlap");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    gg_plan* p = const_cast<gg_plan*>(pc);
    gg::ExecCtx x = fused_ctx(p, stream);
    hipError_t e;
    if (p->dtype == GG_F64) {
        auto v = view<double>(p);
        v.amp_scale = amp_scale;
        e = gg::Ops<double>::make_ic_from_noise(v, static_cast<const double*>(w), pos, vel,
                                                static_cast<double*>(psi_opt), static_cast<gg::cx<double>*>(work), x);
    } else {
        auto v = view<float>(p);
        v.amp_scale = amp_scale;
        e = gg::Ops<float>::make_ic_from_noise(v, static_cast<const float*>(w), pos, vel, static_cast<float*>(psi_opt),
                                               static_cast<gg::cx<float>*>(work), x);
    }
    return e == hipSuccess ? GG_OK : fail_hip(e, "make_ic_from_noise launch");
}

gg_status gg_make_ic_adjoint(const gg_plan* pc, const void* g_psi, const float* g_pos, const float* g_vel,
                             double amp_scale, const void* psi, double* g_log_amp, void* g_w, void* work,
                             void* stream) {
    if (!pc || !g_w || !work) return fail(GG_ERR_INVALID_ARG, "null argument to gg_make_ic_adjoint");
    if (!g_psi && !g_pos && !g_vel) return fail(GG_ERR_INVALID_ARG, "no gradient given (g_psi, g_pos, g_vel)");
    if (g_log_amp && !psi) return fail(GG_ERR_INVALID_ARG, "g_log_amp needs the forward displacements psi");
    if (!(amp_scale > 0) || !std::isfinite(amp_scale)) return fail(GG_ERR_INVALID_ARG, "amp_scale must be > 0");
    if (!aligned(g_w) || !aligned(work) || (g_psi && !aligned(g_psi)) || (g_pos && !aligned(g_pos)) ||
        (g_vel && !aligned(g_vel)) || (psi && !aligned(psi)) || (g_log_amp && ((uintptr_t)g_log_amp & 7u)))
        return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned (g_log_amp 8-byte)");
    const size_t n3 = (size_t)pc->n * pc->n * pc->n;
    const size_t es = elem_size(pc->dtype);
    const size_t wb = gg_workspace_bytes(pc);
    const void* ins[4] = {g_psi, g_pos, g_vel, psi};
    const size_t inb[4] = {3 * es * n3, 12 * n3, 12 * n3, 3 * es * n3};
    for (int i = 0; i < 4; ++i)
        if (ins[i] && (overlap(ins[i], inb[i], work, wb) || overlap(ins[i], inb[i], g_w, es * n3)))
            return fail(GG_ERR_INVALID_ARG, "inputs must not overlap g_w or work");
    if (overlap(g_w, es * n3, work, wb)) return fail(GG_ERR_INVALID_ARG, "g_w must not overlap work");
    if (g_log_amp && overlap(g_log_amp, 8, work, wb)) return fail(GG_ERR_INVALID_ARG, "g_log_amp inside work");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (pc->dtype == GG_F64) {
        auto v = view<double>(pc);
        v.amp_scale = amp_scale;
        e = gg::Ops<double>::adjoint(v, static_cast<const double*>(g_psi), g_pos, g_vel, static_cast<const double*>(psi),
                                     g_log_amp, static_cast<double*>(g_w), static_cast<gg::cx<double>*>(work), s);
    } else {
        auto v = view<float>(pc);
        v.amp_scale = amp_scale;
        e = gg::Ops<float>::adjoint(v, static_cast<const float*>(g_psi), g_pos, g_vel, static_cast<const float*>(psi),
                                    g_log_amp, static_cast<float*>(g_w), static_cast<gg::cx<float>*>(work), s);
    }
    return e == hipSuccess ? GG_OK : fail_hip(e, "make_ic_adjoint launch");
}

gg_status gg_make_density(const gg_plan* pc, uint64_t seed, const void* w_opt, void* delta, void* work,
                          void* stream) {
    if (!pc || !delta || !work) return fail(GG_ERR_INVALID_ARG, "null argument to gg_make_density");
    if (!aligned(delta) || !aligned(work) || (w_opt && !aligned(w_opt)))
        return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t rb = (size_t)pc->n * pc->n * pc->n * elem_size(pc->dtype);
    const size_t wb = gg_workspace_bytes(pc);
    if (overlap(delta, rb, work, wb) || (w_opt && (overlap(w_opt, rb, work, wb) || overlap(w_opt, rb, delta, rb))))
        return fail(GG_ERR_INVALID_ARG, "delta, w_opt and work must not overlap");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e =
        pc->dtype == GG_F64
            ? gg::Ops<double>::density(view<double>(pc), seed, static_cast<const double*>(w_opt),
                                       static_cast<double*>(delta), static_cast<gg::cx<double>*>(work), s)
            : gg::Ops<float>::density(view<float>(pc), seed, static_cast<const float*>(w_opt), static_cast<float*>(delta),
                                      static_cast<gg::cx<float>*>(work), s);
    return e == hipSuccess ? GG_OK : fail_hip(e, "make_density launch");
}

gg_status gg_power_spectrum(const gg_plan* pc, const void* field, int32_t nbins, double* pk, double* kmean,
                            double* counts, void* work, void* stream) {
    if (!pc || !field || !pk || !kmean || !counts || !work)
        return fail(GG_ERR_INVALID_ARG, "null argument to gg_power_spectrum");
    if (nbins < 1 || nbins > gg::kPkMaxBins) return fail(GG_ERR_INVALID_ARG, "nbins must be in [1, 1024]");
    if (!aligned(field) || !aligned(work) || ((uintptr_t)pk & 7u) || ((uintptr_t)kmean & 7u) || ((uintptr_t)counts & 7u))
        return fail(GG_ERR_INVALID_ARG, "field and work must be 256-byte aligned, outputs 8-byte aligned");
    const size_t rb = (size_t)pc->n * pc->n * pc->n * elem_size(pc->dtype);
    const size_t wb = gg_workspace_bytes(pc);
    const size_t ob = (size_t)nbins * sizeof(double);
    if (overlap(field, rb, work, wb) || overlap(pk, ob, work, wb) || overlap(kmean, ob, work, wb) ||
        overlap(counts, ob, work, wb) || overlap(pk, ob, kmean, ob) || overlap(pk, ob, counts, ob) ||
        overlap(kmean, ob, counts, ob))
        return fail(GG_ERR_INVALID_ARG, "field, outputs and work must not overlap");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e =
        pc->dtype == GG_F64
            ? gg::Ops<double>::power_spectrum(view<double>(pc), static_cast<const double*>(field), nbins, pk, kmean,
                                              counts, static_cast<gg::cx<double>*>(work), wb, s)
            : gg::Ops<float>::power_spectrum(view<float>(pc), static_cast<const float*>(field), nbins, pk, kmean, counts,
                                             static_cast<gg::cx<float>*>(work), wb, s);
    if (e == hipErrorInvalidValue) return fail(GG_ERR_INVALID_ARG, "workspace too small for the requested bins");
    return e == hipSuccess ? GG_OK : fail_hip(e, "power_spectrum launch");
}

gg_status gg_field_stats(const gg_plan* pc, const void* field, double* out, void* work, void* stream) {
    if (!pc || !field || !out || !work) return fail(GG_ERR_INVALID_ARG, "null argument to gg_field_stats");
    if (!aligned(field) || !aligned(work) || ((uintptr_t)out & 7u))
        return fail(GG_ERR_INVALID_ARG, "field and work must be 256-byte aligned, out 8-byte aligned");
    const uint64_t count = (uint64_t)pc->n * pc->n * pc->n;
    const size_t rb = count * elem_size(pc->dtype);
    const size_t wb = gg_workspace_bytes(pc);
    if (overlap(field, rb, work, wb) || overlap(out, 4 * sizeof(double), work, wb) ||
        overlap(out, 4 * sizeof(double), field, rb))
        return fail(GG_ERR_INVALID_ARG, "field, out and work must not overlap");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    const size_t fit = wb / (3 * sizeof(double));
    const int nblocks = (int)(fit < 1024 ? fit : 1024);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* scratch = static_cast<double*>(work);
    const hipError_t e =
        pc->dtype == GG_F64
            ? gg::Ops<double>::field_stats(static_cast<const double*>(field), count, out, scratch, nblocks, s)
            : gg::Ops<float>::field_stats(static_cast<const float*>(field), count, out, scratch, nblocks, s);
    return e == hipSuccess ? GG_OK : fail_hip(e, "field_stats launch");
}

gg_status gg_refine_noise_region(int32_t n_parent, const int32_t origin[3], int32_t count, gg_dtype dtype,
                                 gg_refine variant, const void* parent, uint64_t seed, uint32_t stream_id, void* child,
                                 void* stream) {
    if (!parent || !child || !origin) return fail(GG_ERR_INVALID_ARG, "null argument to gg_refine_noise_region");
    if (!valid_dtype(dtype)) return fail(GG_ERR_INVALID_ARG, "unknown dtype");
    int nl = 0, nh = 0;
    gg::refine_sizes(enum_bits(variant), nl, nh);
    if (nl == 0) return fail(GG_ERR_INVALID_ARG, "unknown refinement variant");
    if (n_parent < 1 || n_parent > 4096) return fail(GG_ERR_INVALID_ARG, "n_parent must be in [1, 4096]");
    if (count < nl || count % nl || count > n_parent)
        return fail(GG_ERR_INVALID_ARG, "count must be a positive multiple of N_L, at most n_parent");
    for (int a = 0; a < 3; ++a)
        if (origin[a] < 0 || origin[a] >= n_parent) return fail(GG_ERR_INVALID_ARG, "origin must be in [0, n_parent)");
    if (!aligned(parent) || !aligned(child)) return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t es = elem_size(dtype);
    const size_t nc = (size_t)count / nl * nh;
    if (overlap(parent, (size_t)n_parent * n_parent * n_parent * es, child, nc * nc * nc * es))
        return fail(GG_ERR_INVALID_ARG, "parent and child must not overlap");
    const int o[3] = {origin[0], origin[1], origin[2]};
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = dtype == GG_F64
                             ? gg::Ops<double>::refine((int)variant, static_cast<const double*>(parent), n_parent, o,
                                                       count, seed, stream_id, static_cast<double*>(child), s)
                             : gg::Ops<float>::refine((int)variant, static_cast<const float*>(parent), n_parent, o, count,
                                                      seed, stream_id, static_cast<float*>(child), s);
    return e == hipSuccess ? GG_OK : fail_hip(e, "refine launch");
}

gg_status gg_refine_noise(int32_t n_parent, gg_dtype dtype, gg_refine variant, const void* parent, uint64_t seed,
                          uint32_t stream_id, void* child, void* stream) {
    if (!valid_dtype(dtype)) return fail(GG_ERR_INVALID_ARG, "unknown dtype");
    int nl = 0, nh = 0;
    gg::refine_sizes(enum_bits(variant), nl, nh);
    if (nl == 0) return fail(GG_ERR_INVALID_ARG, "unknown refinement variant");
    if (n_parent < nl || n_parent % nl) return fail(GG_ERR_INVALID_ARG, "n_parent must be a positive multiple of N_L");
    const int32_t origin[3] = {0, 0, 0};
    return gg_refine_noise_region(n_parent, origin, n_parent, dtype, variant, parent, seed, stream_id, child, stream);
}

gg_status gg_make_displacements(const gg_plan* pc, const void* w, int64_t n2_min, int64_t n2_max,
                                int32_t cic_deconvolve, void* psi, void* work, void* stream) {
    if (!pc || !w || !psi || !work) return fail(GG_ERR_INVALID_ARG, "null argument to gg_make_displacements");
    if (n2_min < 0) return fail(GG_ERR_INVALID_ARG, "n2_min must be >= 0");
    if (!aligned(w) || !aligned(psi) || !aligned(work)) return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t es = elem_size(pc->dtype);
    const size_t n3 = (size_t)pc->n * pc->n * pc->n;
    const size_t wb = gg_workspace_bytes(pc);
    if (overlap(w, es * n3, work, wb) || overlap(psi, 3 * es * n3, work, wb) || overlap(psi, 3 * es * n3, w, es * n3))
        return fail(GG_ERR_INVALID_ARG, "w, psi and work must not overlap");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    const int64_t big = 0x7FFFFFFF;
    const int lo = (int)(n2_min < big ? n2_min : big);
    const int hi = (int)(n2_max <= 0 || n2_max > big ? big : n2_max);
    gg_plan* p = const_cast<gg_plan*>(pc);
    gg::ExecCtx x = fused_ctx(p, stream);
    hipError_t e;
    if (p->dtype == GG_F64) {
        auto v = view<double>(p);
        v.n2_lo = lo;
        v.n2_hi = hi;
        v.deconv = cic_deconvolve ? 1 : 0;
        e = gg::Ops<double>::make_ic_from_noise(v, static_cast<const double*>(w), nullptr, nullptr, static_cast<double*>(psi),
                                                static_cast<gg::cx<double>*>(work), x);
    } else {
        auto v = view<float>(p);
        v.n2_lo = lo;
        v.n2_hi = hi;
        v.deconv = cic_deconvolve ? 1 : 0;
        e = gg::Ops<float>::make_ic_from_noise(v, static_cast<const float*>(w), nullptr, nullptr, static_cast<float*>(psi),
                                               static_cast<gg::cx<float>*>(work), x);
    }
    return e == hipSuccess ? GG_OK : fail_hip(e, "make_displacements launch");
}

namespace {

// dst += CiC interpolation of src at origin + m num / den source cells (validated sizes)
gg_status interpolate_add_step(int32_t n_src, int32_t num, int32_t den, const int32_t origin[3], int32_t n_dst,
                               gg_dtype dtype, const void* src, void* dst, void* stream) {
    for (int a = 0; a < 3; ++a)
        if (origin[a] < 0 || origin[a] >= n_src) return fail(GG_ERR_INVALID_ARG, "origin must be in [0, n_src)");
    if (!aligned(src) || !aligned(dst)) return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t es = elem_size(dtype);
    if (overlap(src, 3 * es * n_src * (size_t)n_src * n_src, dst, 3 * es * n_dst * (size_t)n_dst * n_dst))
        return fail(GG_ERR_INVALID_ARG, "src and dst must not overlap");
    const int o[3] = {origin[0], origin[1], origin[2]};
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e =
        dtype == GG_F64 ? gg::Ops<double>::cic_add(static_cast<const double*>(src), n_src, num, den, o,
                                                   static_cast<double*>(dst), n_dst, s)
                        : gg::Ops<float>::cic_add(static_cast<const float*>(src), n_src, num, den, o,
                                                  static_cast<float*>(dst), n_dst, s);
    return e == hipSuccess ? GG_OK : fail_hip(e, "interpolate_add launch");
}

}  // namespace

gg_status gg_interpolate_add_at(int32_t n_src, int32_t ratio, const int32_t origin[3], int32_t n_dst, gg_dtype dtype,
                                const void* src, void* dst, void* stream) {
    if (!src || !dst || !origin) return fail(GG_ERR_INVALID_ARG, "null argument to gg_interpolate_add_at");
    if (!valid_dtype(dtype)) return fail(GG_ERR_INVALID_ARG, "unknown dtype");
    if (n_src < 1 || n_src > 4096 || n_dst < 1 || n_dst > 4096 || ratio < 1 || ratio > 64)
        return fail(GG_ERR_INVALID_ARG, "sizes in [1, 4096], ratio in [1, 64]");
    return interpolate_add_step(n_src, 1, ratio, origin, n_dst, dtype, src, dst, stream);
}

gg_status gg_interpolate_add(int32_t n_src, int32_t n_dst, gg_dtype dtype, const void* src, void* dst, void* stream) {
    if (!src || !dst) return fail(GG_ERR_INVALID_ARG, "null argument to gg_interpolate_add");
    if (!valid_dtype(dtype)) return fail(GG_ERR_INVALID_ARG, "unknown dtype");
    if (n_src < 1 || n_src > 4096 || n_dst < n_src || n_dst > 4096)
        return fail(GG_ERR_INVALID_ARG, "sizes must satisfy 1 <= n_src <= n_dst <= 4096");
    int32_t a = n_src, b = n_dst;
    while (b) {
        const int32_t r = a % b;
        a = b;
        b = r;
    }
    const int32_t origin[3] = {0, 0, 0};
    return interpolate_add_step(n_src, n_src / a, n_dst / a, origin, n_dst, dtype, src, dst, stream);
}

int64_t gg_cutoff_n2(double box, double r_s) {
    if (!(box > 0) || !(r_s > 0) || !std::isfinite(box) || !std::isfinite(r_s)) return -1;
    const double t = box / (2.0 * 3.14159265358979323846 * r_s);
    const double c = std::ceil(t * t);
    return c < 9.0e18 ? (int64_t)c : INT64_MAX;
}

gg_status gg_increase_resolution(const gg_plan* parent, const gg_plan* child, const void* w_parent, gg_refine variant,
                                 uint64_t seed, uint32_t stream_id, double r_s, void* w_child, void* psi, void* work,
                                 void* stream) {
    if (!parent || !child || !w_parent || !w_child || !psi || !work)
        return fail(GG_ERR_INVALID_ARG, "null argument to gg_increase_resolution");
    if (parent->dtype != child->dtype) return fail(GG_ERR_INVALID_ARG, "parent and child plans must share the dtype");
    if (parent->box != child->box) return fail(GG_ERR_INVALID_ARG, "parent and child plans must cover the same box");
    int nl = 0, nh = 0;
    gg::refine_sizes(enum_bits(variant), nl, nh);
    if (nl == 0) return fail(GG_ERR_INVALID_ARG, "unknown refinement variant");
    if (parent->n % nl || parent->n / nl * nh != child->n)
        return fail(GG_ERR_INVALID_ARG, "the child lattice must have n_parent N_H / N_L cells per side");
    if (!(r_s >= 0) || !std::isfinite(r_s)) return fail(GG_ERR_INVALID_ARG, "r_s must be >= 0 (0: two parent cells)");
    if (!aligned(w_parent) || !aligned(w_child) || !aligned(psi) || !aligned(work))
        return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t es = elem_size(parent->dtype);
    const size_t np3 = (size_t)parent->n * parent->n * parent->n;
    const size_t nc3 = (size_t)child->n * child->n * child->n;
    const size_t wb = gg_workspace_bytes(child);
    // the parent's large-scale fields, then the parent's transform workspace,
    // both inside the child's workspace (free once Eq. 4 is done)
    const size_t large_bytes = (3 * es * np3 + 255) & ~(size_t)255;
    if (large_bytes + gg_workspace_bytes(parent) > wb)
        return fail(GG_ERR_INTERNAL, "child workspace cannot hold the parent's fields");
    if (overlap(w_parent, es * np3, w_child, es * nc3) || overlap(w_parent, es * np3, psi, 3 * es * nc3) ||
        overlap(w_parent, es * np3, work, wb) || overlap(w_child, es * nc3, psi, 3 * es * nc3) ||
        overlap(w_child, es * nc3, work, wb) || overlap(psi, 3 * es * nc3, work, wb))
        return fail(GG_ERR_INVALID_ARG, "w_parent, w_child, psi and work must not overlap");
    gg_status st = check_device(parent);
    if (st == GG_OK) st = check_device(child);
    if (st != GG_OK) return st;
    const int64_t cut = gg_cutoff_n2(parent->box, r_s > 0 ? r_s : 2.0 * parent->cell);
    void* large = work;
    void* pwork = static_cast<char*>(work) + large_bytes;
    st = gg_refine_noise(parent->n, parent->dtype, variant, w_parent, seed, stream_id, w_child, stream);
    if (st == GG_OK) st = gg_make_displacements(child, w_child, cut, 0, 0, psi, work, stream);
    if (st == GG_OK) st = gg_make_displacements(parent, w_parent, 0, cut, 1, large, pwork, stream);
    if (st == GG_OK) st = gg_interpolate_add(parent->n, child->n, parent->dtype, large, psi, stream);
    return st;
}

gg_status gg_lowpass(const gg_plan* pc, const void* field, int64_t n2_max, int32_t cic_deconvolve, void* out, void* work,
                     void* stream) {
    if (!pc || !field || !out || !work) return fail(GG_ERR_INVALID_ARG, "null argument to gg_lowpass");
    if (!aligned(field) || !aligned(out) || !aligned(work)) return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t rb = (size_t)pc->n * pc->n * pc->n * elem_size(pc->dtype);
    const size_t wb = gg_workspace_bytes(pc);
    if (overlap(field, rb, work, wb) || overlap(out, rb, work, wb))
        return fail(GG_ERR_INVALID_ARG, "field, out and work must not overlap (field may equal out)");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    const int hi = (int)(n2_max <= 0 || n2_max > 0x7FFFFFFF ? 0x7FFFFFFF : n2_max);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e =
        pc->dtype == GG_F64
            ? gg::Ops<double>::lowpass(view<double>(pc), static_cast<const double*>(field), hi, cic_deconvolve ? 1 : 0,
                                       static_cast<double*>(out), static_cast<gg::cx<double>*>(work), s)
            : gg::Ops<float>::lowpass(view<float>(pc), static_cast<const float*>(field), hi, cic_deconvolve ? 1 : 0,
                                      static_cast<float*>(out), static_cast<gg::cx<float>*>(work), s);
    return e == hipSuccess ? GG_OK : fail_hip(e, "lowpass launch");
}

gg_status gg_degrade(const gg_plan* pc, const void* fine, int32_t factor, const double shift[3], void* out, void* work,
                     void* stream) {
    if (!pc || !fine || !shift || !out || !work) return fail(GG_ERR_INVALID_ARG, "null argument to gg_degrade");
    if (factor < 1 || factor > kMaxDegrade) return fail(GG_ERR_INVALID_ARG, "factor must be in [1, 16]");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(shift[a]) || std::fabs(shift[a]) > 1e6)
            return fail(GG_ERR_INVALID_ARG, "shift must be finite (|shift| <= 1e6 cells)");
    if (!aligned(fine) || !aligned(out) || !aligned(work)) return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t es = elem_size(pc->dtype);
    const size_t rb = (size_t)pc->n * pc->n * pc->n * es;
    const size_t nf = (size_t)pc->n * factor;
    const size_t fb = nf * nf * nf * es;
    const size_t wb = gg_workspace_bytes(pc);
    if (overlap(fine, fb, out, rb) || overlap(fine, fb, work, wb) || overlap(out, rb, work, wb))
        return fail(GG_ERR_INVALID_ARG, "fine, out and work must not overlap");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e =
        pc->dtype == GG_F64
            ? gg::Ops<double>::degrade(view<double>(pc), static_cast<const double*>(fine), factor, shift,
                                       static_cast<double*>(out), static_cast<gg::cx<double>*>(work), s)
            : gg::Ops<float>::degrade(view<float>(pc), static_cast<const float*>(fine), factor, shift,
                                      static_cast<float*>(out), static_cast<gg::cx<float>*>(work), s);
    return e == hipSuccess ? GG_OK : fail_hip(e, "degrade launch");
}

gg_status gg_zeldovich_at(const gg_plan* pc, const void* psi, const double origin[3], double wrap_box, float* pos,
                          float* vel, void* stream) {
    if (!pc || !psi || !pos || !vel || !origin) return fail(GG_ERR_INVALID_ARG, "null argument to gg_zeldovich_at");
    if (!(wrap_box > 0) || !std::isfinite(wrap_box)) return fail(GG_ERR_INVALID_ARG, "wrap_box must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!(origin[a] >= 0 && origin[a] < wrap_box)) return fail(GG_ERR_INVALID_ARG, "origin must be in [0, wrap_box)");
    if (!aligned(psi) || !aligned(pos) || !aligned(vel)) return fail(GG_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
    const size_t n3 = (size_t)pc->n * pc->n * pc->n;
    if (overlap(pos, 12 * n3, vel, 12 * n3) || overlap(psi, 3 * n3 * elem_size(pc->dtype), pos, 12 * n3) ||
        overlap(psi, 3 * n3 * elem_size(pc->dtype), vel, 12 * n3))
        return fail(GG_ERR_INVALID_ARG, "psi, pos and vel must not overlap");
    gg_status st = check_device(pc);
    if (st != GG_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (pc->dtype == GG_F64) {
        auto v = view<double>(pc);
        for (int a = 0; a < 3; ++a) v.origin[a] = origin[a];
        v.wrap = wrap_box;
        e = gg::Ops<double>::zeldovich(v, static_cast<const double*>(psi), pos, vel, s);
    } else {
        auto v = view<float>(pc);
        for (int a = 0; a < 3; ++a) v.origin[a] = origin[a];
        v.wrap = wrap_box;
        e = gg::Ops<float>::zeldovich(v, static_cast<const float*>(psi), pos, vel, s);
    }
    return e == hipSuccess ? GG_OK : fail_hip(e, "zeldovich launch");
}

namespace {

bool chunks_valid(const gg_plan* p, int c) {
    const int cblocks = (p->n / 2) / (p->dtype == GG_F64 ? gg::Tile<double>::L : gg::Tile<float>::L);
    return c == 1 || (c >= 1 && c <= kMaxChunks && p->n >= 256 && p->aux && (p->n / 8) % c == 0 && cblocks % c == 0);
}

bool lines_valid(const gg_plan* p, int l) {
    if (l == 0) return true;
    int full = 0, half = 0, p1d = 0, zd = 0;
    if (p->dtype == GG_F64) gg::Ops<double>::tile_options(p->n, full, half, p1d, zd);
    else gg::Ops<float>::tile_options(p->n, full, half, p1d, zd);
    return l == full || l == half;
}

}  // namespace

gg_status gg_plan_set_tuning(gg_plan* p, int32_t chunks, int32_t p1_lines, int32_t z_lines) {
    if (!p) return fail(GG_ERR_INVALID_ARG, "null plan");
    if (chunks != 0 && !chunks_valid(p, chunks)) return fail(GG_ERR_INVALID_ARG, "chunk count not valid for this lattice");
    if (!lines_valid(p, p1_lines) || !lines_valid(p, z_lines))
        return fail(GG_ERR_INVALID_ARG, "lines must be 0 or the full or half LDS row of lines");
    if (chunks != 0) p->nchunk = chunks;
    p->p1_lines = p1_lines;
    p->z_lines = z_lines;
    return GG_OK;
}

// relative speed-up a later autotuner candidate needs to replace the best so far
constexpr double kTuneMargin = 0.005;

gg_status gg_plan_autotune(gg_plan* p, float* pos, float* vel, void* work, int32_t reps, gg_tune_entry* results,
                           int32_t capacity, int32_t* count, void* stream) {
    if (!p || !pos || !vel || !work || !count) return fail(GG_ERR_INVALID_ARG, "null argument to gg_plan_autotune");
    if (reps < 1 || reps > 100) return fail(GG_ERR_INVALID_ARG, "reps must be in [1, 100]");
    if (p->timing) return fail(GG_ERR_INVALID_ARG, "disable timing before autotuning");
    int full = 0, half = 0, p1d = 0, zd = 0;
    if (p->dtype == GG_F64) gg::Ops<double>::tile_options(p->n, full, half, p1d, zd);
    else gg::Ops<float>::tile_options(p->n, full, half, p1d, zd);
    std::vector<int> chunk_set, lines_set{full};
    if (half != full) lines_set.push_back(half);
    for (int c = 1; c <= kMaxChunks; c *= 2)
        if (chunks_valid(p, c)) chunk_set.push_back(c);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) {
        if (t0) (void)hipEventDestroy(t0);
        return fail_hip(e, "hipEventCreate");
    }
    const int keep_c = p->nchunk, keep_1 = p->p1_lines, keep_z = p->z_lines;
    double best = 1e300;
    int bc = keep_c, b1 = keep_1, bz = keep_z;
    int n = 0;
    gg_status st = GG_OK;
    for (int c : chunk_set)
        for (int l1 : lines_set)
            for (int lz : lines_set) {
                p->nchunk = c;
                p->p1_lines = l1;
                p->z_lines = lz;
                st = gg_make_ic(p, 0, pos, vel, nullptr, work, stream);  // warm-up
                if (st != GG_OK) break;
                if ((e = hipEventRecord(t0, s)) != hipSuccess) break;
                for (int r = 0; r < reps && st == GG_OK; ++r) st = gg_make_ic(p, (uint64_t)r + 1, pos, vel, nullptr, work, stream);
                if (st != GG_OK) break;
                if ((e = hipEventRecord(t1, s)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess) break;
                float ms = 0.f;
                if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
                const double per = (double)ms / reps;
                if (results && n < capacity) results[n] = gg_tune_entry{c, l1, lz, per};
                ++n;
                // a later configuration (more chunks, narrower tiles) must win by
                // more than the timing noise, so that near-ties keep the simpler
                // one and repeated tuning settles on the same choice
                if (per < best * (1.0 - kTuneMargin)) {
                    best = per;
                    bc = c;
                    b1 = l1;
                    bz = lz;
                }
            }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (st != GG_OK || e != hipSuccess) {
        p->nchunk = keep_c;
        p->p1_lines = keep_1;
        p->z_lines = keep_z;
        return st != GG_OK ? st : fail_hip(e, "autotune timing");
    }
    p->nchunk = bc;
    p->p1_lines = b1;
    p->z_lines = bz;
    *count = n;
    return GG_OK;
}

gg_status gg_timing_enable(gg_plan* p, int on) {
    if (!p) return fail(GG_ERR_INVALID_ARG, "null plan");
    if (on && p->events.empty()) {
        p->events.resize((size_t)kTimingSlots * 2 * kLaunchesMax);
        for (auto& ev : p->events) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return fail_hip(e, "hipEventCreate");
        }
    }
    p->timing = on != 0;
    p->recorded = 0;
    return GG_OK;
}

gg_status gg_timing_read(gg_plan* p, double* ms, int npass, int* ncalls) {
    if (!p || !ms || !ncalls) return fail(GG_ERR_INVALID_ARG, "null argument to gg_timing_read");
    if (npass != kPasses) return fail(GG_ERR_INVALID_ARG, "npass must be 5");
    for (int i = 0; i < npass; ++i) ms[i] = 0;
    *ncalls = p->recorded;
    if (p->recorded == 0) return GG_OK;
    const int nc = p->nchunk;
    const int launches = 4 * nc + 1;
    hipError_t e = hipEventSynchronize(p->events[(size_t)(p->recorded - 1) * 2 * kLaunchesMax + 2 * launches - 1]);
    if (e != hipSuccess) return fail_hip(e, "hipEventSynchronize");
    for (int r = 0; r < p->recorded; ++r) {
        const hipEvent_t* ev = &p->events[(size_t)r * 2 * kLaunchesMax];
        for (int k = 0; k < launches; ++k) {
            float t = 0;
            e = hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]);
            if (e != hipSuccess) return fail_hip(e, "hipEventElapsedTime");
            ms[k / nc < kPasses ? k / nc : kPasses - 1] += t;
        }
    }
    p->recorded = 0;
    return GG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Zoom hierarchy (Sec. 2.3-2.4): one plan per level, run on the caller's
// stream and two streams of the hierarchy ordered by events, optionally
// captured once into a HIP graph and replayed.
// ---------------------------------------------------------------------------
struct gg_zoom {
    gg_zoom_desc d{};
    gg_dtype dtype = GG_F32;
    std::vector<gg_plan*> plans;
    std::vector<double> box, cell;
    std::vector<std::array<double, 3>> origin_box;  // level origin in the base box
    size_t plan_work = 0;                           // max plan workspace
    size_t tmp_bytes = 0;                           // 3 R of the largest parent
    // the hierarchy runs as three streams: the caller's (base noise and base
    // particles), side[0] (noise refinement and Eq. 4 of every level, which
    // depend on the noise only) and side[1] (the chain of Eq. 5 and the CiC
    // interpolation with the level's particles, level by level); events order
    // them
    hipStream_t side[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> ev;  // kZoomEvents
    // workspace layout (bytes from the start): the chain's transform work and
    // the parent's filtered fields, then one transform work per level for its
    // Eq. 4 (level 0: the base particles)
    size_t chain_off = 0, tmp_off = 0;
    std::vector<size_t> level_off;
    size_t total_work = 0;
    // captured graph and the arguments it was captured with
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> key;
    uint64_t key_seed = 0;
};

namespace {

// events per hierarchy: base noise done, Eq. 4 of level l done (8), the two
// side streams done (2)
constexpr int kZoomEvents = 1 + GG_ZOOM_MAX_LEVELS + 2;
constexpr int kEvW0 = 0;
constexpr int kEvEq4 = 1;
constexpr int kEvEnd = 1 + GG_ZOOM_MAX_LEVELS;

void zoom_free(gg_zoom* z) {
    if (!z) return;
    if (z->exec) (void)hipGraphExecDestroy(z->exec);
    if (z->graph) (void)hipGraphDestroy(z->graph);
    for (hipEvent_t e : z->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t st : z->side)
        if (st) (void)hipStreamDestroy(st);
    for (gg_plan* p : z->plans) gg_plan_destroy(p);
    delete z;
}

}  // namespace

gg_status gg_zoom_create(gg_zoom** out, const gg_zoom_desc* d, const gg_cosmo* cosmo, gg_dtype dtype) {
    if (!out || !d || !cosmo) return fail(GG_ERR_INVALID_ARG, "null argument to gg_zoom_create");
    if (!valid_dtype(dtype)) return fail(GG_ERR_INVALID_ARG, "dtype must be GG_F32 or GG_F64");
    if (d->levels < 1 || d->levels > GG_ZOOM_MAX_LEVELS) return fail(GG_ERR_INVALID_ARG, "levels must be in [1, 8]");
    if (!(d->box > 0) || !std::isfinite(d->box)) return fail(GG_ERR_INVALID_ARG, "box must be > 0");
    int nl = 0, nh = 0;
    gg::refine_sizes((int)d->variant, nl, nh);
    if (nl == 0 || nh != 2 * nl) return fail(GG_ERR_INVALID_ARG, "zoom levels refine by two: variant HR, 4, LINEAR or SINE");
    for (int l = 0; l < d->levels; ++l) {
        if (!gg::supported_n(d->n[l])) return fail(GG_ERR_UNSUPPORTED_SIZE, "unsupported level size");
        if (l > 0) {
            const int span = d->n[l] / 2;
            if (d->n[l] % (2 * nl) || span > d->n[l - 1])
                return fail(GG_ERR_INVALID_ARG, "a level spans n/2 parent cells (a multiple of N_L, within the parent)");
            for (int a = 0; a < 3; ++a) {
                const int o = d->origin[l][a];
                if (o < 0 || o >= d->n[l - 1]) return fail(GG_ERR_INVALID_ARG, "origin outside the parent lattice");
                // levels below the first sit inside their parent's sub-box (no wrap)
                if (l > 1 && o + span > d->n[l - 1])
                    return fail(GG_ERR_INVALID_ARG, "a nested level must lie inside its parent sub-box");
            }
        }
    }
    gg_zoom* z = new (std::nothrow) gg_zoom;
    if (!z) return fail(GG_ERR_OUT_OF_MEMORY, "zoom");
    z->d = *d;
    z->dtype = dtype;
    const size_t es = elem_size(dtype);
    double cell = d->box / d->n[0];
    std::array<double, 3> org{0.0, 0.0, 0.0};
    for (int l = 0; l < d->levels; ++l) {
        if (l > 0) {
            for (int a = 0; a < 3; ++a) org[a] = std::fmod(org[a] + d->origin[l][a] * cell, d->box);
            cell *= 0.5;
        }
        const double box = d->n[l] * cell;
        gg_grid g{d->n[l], box};
        gg_plan* p = nullptr;
        gg_status st = gg_plan_create(&p, &g, cosmo, dtype);
        if (st != GG_OK) {
            zoom_free(z);
            return st;
        }
        p->nchunk = 1;  // no plan-owned stream: the hierarchy's own streams are the whole schedule
        z->plans.push_back(p);
        z->box.push_back(box);
        z->cell.push_back(cell);
        z->origin_box.push_back(org);
        z->plan_work = std::max(z->plan_work, gg_workspace_bytes(p));
        if (l + 1 < d->levels) z->tmp_bytes = std::max(z->tmp_bytes, 3 * es * (size_t)d->n[l] * d->n[l] * d->n[l]);
    }
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    z->chain_off = 0;
    z->tmp_off = up(z->plan_work);
    size_t off = z->tmp_off + up(z->tmp_bytes);
    for (int l = 0; l < d->levels; ++l) {
        z->level_off.push_back(off);
        off += up(gg_workspace_bytes(z->plans[l]));
    }
    z->total_work = off;
    hipError_t e = hipSuccess;
    for (hipStream_t& st : z->side)
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    z->ev.assign(kZoomEvents, nullptr);
    for (hipEvent_t& ev : z->ev)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        zoom_free(z);
        return fail_hip(e, "zoom streams and events");
    }
    *out = z;
    return GG_OK;
}

gg_status gg_zoom_destroy(gg_zoom* z) {
    if (!z) return GG_OK;
    if (!z->plans.empty()) (void)hipSetDevice(z->plans[0]->device);
    (void)hipDeviceSynchronize();
    zoom_free(z);
    return GG_OK;
}

size_t gg_zoom_workspace_bytes(const gg_zoom* z) {
    if (!z) return 0;
    return z->total_work;
}

gg_status gg_zoom_autotune(gg_zoom* z, uint64_t seed, void* const* w, void* const* psi, float* const* pos,
                           float* const* vel, void* work, int32_t reps, gg_zoom_tune_entry* results, int32_t capacity,
                           int32_t* count, void* stream) {
    if (!z || !count) return fail(GG_ERR_INVALID_ARG, "null argument to gg_zoom_autotune");
    if (reps < 1 || reps > 100) return fail(GG_ERR_INVALID_ARG, "reps must be in [1, 100]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) {
        if (t0) (void)hipEventDestroy(t0);
        return fail_hip(e, "hipEventCreate");
    }
    auto time_run = [&](double& ms_out) -> gg_status {
        gg_status st = gg_zoom_run(z, seed, w, psi, pos, vel, work, 0, stream);  // warm-up
        if (st != GG_OK) return st;
        if ((e = hipEventRecord(t0, s)) != hipSuccess) return fail_hip(e, "autotune timing");
        for (int r = 0; r < reps && st == GG_OK; ++r) st = gg_zoom_run(z, seed, w, psi, pos, vel, work, 0, stream);
        if (st != GG_OK) return st;
        if ((e = hipEventRecord(t1, s)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess)
            return fail_hip(e, "autotune timing");
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) return fail_hip(e, "autotune timing");
        ms_out = (double)ms / reps;
        return GG_OK;
    };
    // one level at a time (the others at their current choice): the tile
    // widths of its first and last fused passes, full LDS row or half; a later
    // choice must win by the same margin as in gg_plan_autotune
    int n = 0;
    gg_status st = GG_OK;
    for (int l = 0; l < z->d.levels && st == GG_OK; ++l) {
        gg_plan* p = z->plans[l];
        int full = 0, half = 0, p1d = 0, zd = 0;
        if (p->dtype == GG_F64) gg::Ops<double>::tile_options(p->n, full, half, p1d, zd);
        else gg::Ops<float>::tile_options(p->n, full, half, p1d, zd);
        std::vector<int> lines_set{full};
        if (half != full) lines_set.push_back(half);
        const int keep_1 = p->p1_lines, keep_z = p->z_lines;
        double best = 1e300;
        int b1 = keep_1, bz = keep_z;
        for (int l1 : lines_set) {
            for (int lz : lines_set) {
                p->p1_lines = l1;
                p->z_lines = lz;
                double ms = 0.0;
                if ((st = time_run(ms)) != GG_OK) break;
                if (results && n < capacity) results[n] = gg_zoom_tune_entry{l, l1, lz, ms};
                ++n;
                if (ms < best * (1.0 - kTuneMargin)) {
                    best = ms;
                    b1 = l1;
                    bz = lz;
                }
            }
            if (st != GG_OK) break;
        }
        p->p1_lines = st == GG_OK ? b1 : keep_1;
        p->z_lines = st == GG_OK ? bz : keep_z;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    // a graph captured before holds the old launch shapes
    if (z->exec) {
        (void)hipGraphExecDestroy(z->exec);
        z->exec = nullptr;
    }
    if (z->graph) {
        (void)hipGraphDestroy(z->graph);
        z->graph = nullptr;
    }
    if (st != GG_OK) return st;
    *count = n;
    return GG_OK;
}

gg_status gg_zoom_query(const gg_zoom* z, int32_t level, double* box, double* cell, double origin[3]) {
    if (!z || !box || !cell || !origin) return fail(GG_ERR_INVALID_ARG, "null argument to gg_zoom_query");
    if (level < 0 || level >= z->d.levels) return fail(GG_ERR_INVALID_ARG, "level out of range");
    *box = z->box[level];
    *cell = z->cell[level];
    for (int a = 0; a < 3; ++a) origin[a] = z->origin_box[level][a];
    return GG_OK;
}

namespace {

// Eq. 5 of the three components of a level's displacements (3 R of plan p)
// into out (3 R): the pruned three-field transform
gg_status zoom_lowpass3(const gg_plan* p, const void* field, int64_t n2_max, void* out, void* work, hipStream_t s) {
    const int hi = (int)(n2_max <= 0 || n2_max > 0x7FFFFFFF ? 0x7FFFFFFF : n2_max);
    const hipError_t e =
        p->dtype == GG_F64
            ? gg::Ops<double>::lowpass3(view<double>(p), static_cast<const double*>(field), hi, 1,
                                        static_cast<double*>(out), static_cast<gg::cx<double>*>(work), s)
            : gg::Ops<float>::lowpass3(view<float>(p), static_cast<const float*>(field), hi, 1, static_cast<float*>(out),
                                       static_cast<gg::cx<float>*>(work), s);
    return e == hipSuccess ? GG_OK : fail_hip(e, "zoom lowpass launch");
}

// Eq. 5 of the base displacements as the base filter on the large-scale
// window (with the CiC deconvolution) applied to the base noise: psi (3 R)
gg_status zoom_base_window(gg_plan* p, const void* w, int64_t n2_max, void* psi, void* work, hipStream_t s) {
    const int hi = (int)(n2_max <= 0 || n2_max > 0x7FFFFFFF ? 0x7FFFFFFF : n2_max);
    const gg::ExecCtx x = fused_ctx(p, s);
    const hipError_t e =
        p->dtype == GG_F64
            ? gg::Ops<double>::windowed_displacements(view<double>(p), static_cast<const double*>(w), hi, 1,
                                                      static_cast<double*>(psi), static_cast<gg::cx<double>*>(work), x)
            : gg::Ops<float>::windowed_displacements(view<float>(p), static_cast<const float*>(w), hi, 1,
                                                     static_cast<float*>(psi), static_cast<gg::cx<float>*>(work), x);
    return e == hipSuccess ? GG_OK : fail_hip(e, "zoom window launch");
}

gg_status zoom_sequence(gg_zoom* z, uint64_t seed, void* const* w, void* const* psi, float* const* pos,
                        float* const* vel, void* work, void* stream) {
    const gg_zoom_desc& d = z->d;
    char* wk = static_cast<char*>(work);
    void* chain = wk + z->chain_off;
    void* tmp = wk + z->tmp_off;
    hipStream_t s0 = static_cast<hipStream_t>(stream);
    hipStream_t s1 = z->side[0], s2 = z->side[1];
    gg_status st;
    hipError_t e;
#define GG_Z(expr) \
    if ((st = (expr)) != GG_OK) return st;
#define GG_ZH(expr) \
    if ((e = (expr)) != hipSuccess) return fail_hip(e, "zoom stream ordering");
    GG_Z(gg_noise(z->plans[0], seed, 0u, w[0], stream))
    GG_ZH(hipEventRecord(z->ev[kEvW0], s0))
    GG_ZH(hipStreamWaitEvent(s1, z->ev[kEvW0], 0))
    GG_ZH(hipStreamWaitEvent(s2, z->ev[kEvW0], 0))
    // the caller's stream: the base particles
    auto base = [&]() -> gg_status {
        return gg_make_ic_from_noise(z->plans[0], w[0], 1.0, pos[0], vel[0], psi[0], wk + z->level_off[0], s0);
    };
    // side[0]: the level's noise (App. A refinement of its parent's sub-box)
    // and its small scales (Eq. 4 on its own periodic sub-box)
    auto small = [&](int l) -> gg_status {
        const int np = d.n[l - 1], n = d.n[l];
        const double r_s = 2.0 * z->cell[l - 1];
        gg_status r = gg_refine_noise_region(np, d.origin[l], n / 2, z->dtype, (gg_refine)d.variant, w[l - 1], seed,
                                             (uint32_t)l, w[l], s1);
        if (r != GG_OK) return r;
        r = gg_make_displacements(z->plans[l], w[l], gg_cutoff_n2(z->box[l], r_s), 0, 0, psi[l], wk + z->level_off[l],
                                  s1);
        if (r != GG_OK) return r;
        const hipError_t he = hipEventRecord(z->ev[kEvEq4 + l], s1);
        return he == hipSuccess ? GG_OK : fail_hip(he, "zoom stream ordering");
    };
    // side[1]: the level's large scales (Eq. 5 of its parent's final
    // displacements), chained from level to level ...
    auto large = [&](int l) -> gg_status {
        const double r_s = 2.0 * z->cell[l - 1];
        if (l == 1) {
            // the base displacements are the filtered base noise, so Eq. 5 of them
            // is that filter on the large-scale window: one fused pass sequence
            // over the base noise instead of three transform round trips
            return zoom_base_window(z->plans[0], w[0], gg_cutoff_n2(z->box[0], r_s), tmp, chain, s2);
        }
        return zoom_lowpass3(z->plans[l - 1], psi[l - 1], gg_cutoff_n2(z->box[l - 1], r_s), tmp, chain, s2);
    };
    // ... CiC-interpolated onto the level once its small scales exist; the
    // same pass writes the level's particles (Eq. 3 at the level's lattice in
    // the base box) from the final displacements
    auto join = [&](int l) -> gg_status {
        hipError_t he = hipStreamWaitEvent(s2, z->ev[kEvEq4 + l], 0);
        if (he != hipSuccess) return fail_hip(he, "zoom stream ordering");
        const gg_plan* pl = z->plans[l];
        const int o[3] = {d.origin[l][0], d.origin[l][1], d.origin[l][2]};
        if (pl->dtype == GG_F64) {
            auto v = view<double>(pl);
            for (int a = 0; a < 3; ++a) v.origin[a] = z->origin_box[l][a];
            v.wrap = d.box;
            he = gg::Ops<double>::cic_add_zel(static_cast<const double*>(tmp), d.n[l - 1], 1, 2, o,
                                              static_cast<double*>(psi[l]), v, pos[l], vel[l], s2);
        } else {
            auto v = view<float>(pl);
            for (int a = 0; a < 3; ++a) v.origin[a] = z->origin_box[l][a];
            v.wrap = d.box;
            he = gg::Ops<float>::cic_add_zel(static_cast<const float*>(tmp), d.n[l - 1], 1, 2, o,
                                             static_cast<float*>(psi[l]), v, pos[l], vel[l], s2);
        }
        return he == hipSuccess ? GG_OK : fail_hip(he, "zoom interpolation launch");
    };
    // Issue order: every level's small scales, then the chain of large scales
    // (with the level particles), then the base particles.  A captured graph
    // keeps this order in how it spreads the branches over hardware queues:
    // issuing the base particles or a level's large scales first measured
    // slower replayed, and no order changed the eager time.
    for (int l = 1; l < d.levels; ++l) GG_Z(small(l))
    for (int l = 1; l < d.levels; ++l) {
        GG_Z(large(l))
        GG_Z(join(l))
    }
    GG_Z(base())
    GG_ZH(hipEventRecord(z->ev[kEvEnd], s1))
    GG_ZH(hipEventRecord(z->ev[kEvEnd + 1], s2))
    GG_ZH(hipStreamWaitEvent(s0, z->ev[kEvEnd], 0))
    GG_ZH(hipStreamWaitEvent(s0, z->ev[kEvEnd + 1], 0))
#undef GG_Z
#undef GG_ZH
    return GG_OK;
}

}  // namespace

gg_status gg_zoom_run(gg_zoom* z, uint64_t seed, void* const* w, void* const* psi, float* const* pos, float* const* vel,
                      void* work, int32_t use_graph, void* stream) {
    if (!z || !w || !psi || !pos || !vel || !work) return fail(GG_ERR_INVALID_ARG, "null argument to gg_zoom_run");
    for (int l = 0; l < z->d.levels; ++l)
        if (!w[l] || !psi[l] || !pos[l] || !vel[l]) return fail(GG_ERR_INVALID_ARG, "null level buffer");
    if (!aligned(work)) return fail(GG_ERR_INVALID_ARG, "work must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!use_graph) return zoom_sequence(z, seed, w, psi, pos, vel, work, stream);
    std::vector<const void*> key;
    for (int l = 0; l < z->d.levels; ++l) {
        key.push_back(w[l]);
        key.push_back(psi[l]);
        key.push_back(pos[l]);
        key.push_back(vel[l]);
    }
    key.push_back(work);
    key.push_back(stream);
    if (!z->exec || key != z->key || seed != z->key_seed) {
        if (z->exec) {
            (void)hipGraphExecDestroy(z->exec);
            z->exec = nullptr;
        }
        if (z->graph) {
            (void)hipGraphDestroy(z->graph);
            z->graph = nullptr;
        }
        if (s == nullptr) return fail(GG_ERR_INVALID_ARG, "graph capture needs a non-null stream");
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail_hip(e, "hipStreamBeginCapture");
        const gg_status st = zoom_sequence(z, seed, w, psi, pos, vel, work, stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (st != GG_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&z->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail_hip(e, "hipGraphInstantiate");
        }
        z->graph = g;
        z->key = key;
        z->key_seed = seed;
    }
    const hipError_t e = hipGraphLaunch(z->exec, s);
    return e == hipSuccess ? GG_OK : fail_hip(e, "hipGraphLaunch");
}
